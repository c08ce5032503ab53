"""Dirichlet layers (Sec. 2.3: velocity conditions imposed by the volume
penalization) on the GPU against the FP64 oracle; with a body, alone, with the
sponge and RK4; ensembles; parameter checks."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_1506_06513_amd as F
import workloads as W

pytestmark = pytest.mark.gpu

L = 4.0


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def _both(n, nu, eta, u0, body, steps, dtype, wall, u_wall, mean_mode=F.FLUSI_MEAN_FIXED, integrator="ab2",
          sponge=None, **ctl):
    p = O.Params(n, L, nu, eta, mean_mode, wall=tuple(wall), u_wall=tuple(u_wall), integrator=integrator,
                 **({} if sponge is None else dict(c_sp=sponge[0], sponge=tuple(sponge[1]))))
    ost, oh = O.run(p, u0, steps, O.StepControl(**ctl), O.Insect.from_dict(body) if body else None)
    P = F.Plan(n, L, nu, eta, dtype)
    P.set_walls(wall, u_wall)
    P.set_integrator(integrator)
    if sponge is not None:
        P.set_sponge(*sponge)
    st = P.new_state(torch.from_numpy(u0))
    h = P.step(st, steps, body, history=True, mean_mode=mean_mode, **ctl).cpu().numpy()
    return O.velocity(p, ost), oh, P.velocity(st).cpu().numpy(), h


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sphere_with_inflow_layer(dtype):
    n = 48
    u0 = W.inflow_noise(n, L, seed=70, rms=1e-2, kmax=6.0)
    ou, oh, u, h = _both(n, 0.01, 1e-3, u0, W.sphere_body(L), 20, dtype, (0.5, 0.0, 0.0), (1.0, 0.0, 0.0), cfl=0.1)
    assert rel_l2(u, ou) < (1e-11 if dtype == "f64" else 2e-5)
    oF = np.array([d["F"][0] for d in oh])
    assert np.max(np.abs(h[:, 4:7] - oF)) <= (1e-10 if dtype == "f64" else 1e-4) * np.max(np.abs(oF))
    odt = np.array([d["dt"] for d in oh])
    assert np.max(np.abs(h[:, 1] - odt)) <= 1e-12 * odt.max()


def test_layers_without_a_body():
    n = 32
    u0 = W.inflow_noise(n, L, seed=71, rms=0.2, kmax=4.0)
    ou, oh, u, h = _both(n, 0.02, 1e-2, u0, None, 15, "f64", (0.5, 0.75, 0.0), (0.5, -0.25, 0.1),
                         mean_mode=F.FLUSI_MEAN_FREE, cfl=0.1)
    assert rel_l2(u, ou) < 1e-11
    assert np.all(h[:, 4:41] == 0.0)  # no body: no force, pose or power records


def test_layers_with_sponge_and_rk4():
    n = 48
    u0 = W.inflow_noise(n, L, seed=72, rms=1e-2, kmax=6.0)
    ou, _, u, _ = _both(n, 0.02, 5e-3, u0, W.sphere_body(L), 5, "f64", (0.25, 0.0, 0.0), (1.0, 0.0, 0.0),
                        integrator="rk4", sponge=(0.1, (0.75, 0.0, 0.0)), cfl=0.1)
    assert rel_l2(u, ou) < 1e-11


def test_mixed_ensemble_and_checks():
    specs = [(48, (0.5, 0.0, 0.0)), (48, None), (32, (0.0, 0.5, 0.5))]
    ens = F.Ensemble("f32")
    pairs = []
    for k, (n, wall) in enumerate(specs):
        u0 = W.inflow_noise(n, L, seed=80 + k, rms=1e-2, kmax=6.0)
        Pa, Pb = F.Plan(n, L, 0.01, 1e-3, "f32"), F.Plan(n, L, 0.01, 1e-3, "f32")
        if wall:
            Pa.set_walls(wall, (1.0, 0.0, 0.0))
            Pb.set_walls(wall, (1.0, 0.0, 0.0))
        sa, sb = Pa.new_state(torch.from_numpy(u0)), Pb.new_state(torch.from_numpy(u0))
        ens.add(Pa, sa, W.model_insect(n, L), cfl=0.1)
        pairs.append((Pa, sa, Pb, sb, n))
    ens.step(3, graph=True)
    for Pa, sa, Pb, sb, n in pairs:
        Pb.step(sb, 3, W.model_insect(n, L), cfl=0.1)
    torch.cuda.synchronize()
    for i, (Pa, sa, Pb, sb, _) in enumerate(pairs):
        assert torch.equal(Pa.uhat(sa), Pb.uhat(sb)), i
    ens.close()
    P = F.Plan(32, L, 0.01, 1e-3, "f32")
    for th, uw in (((-0.1, 0, 0), (1, 0, 0)), ((5.0, 0, 0), (1, 0, 0)), ((0.5, 0, 0), (math.nan, 0, 0))):
        with pytest.raises(F.FlusiError) as e:
            P.set_walls(th, uw)
        assert e.value.code == F.FLUSI_EINVAL

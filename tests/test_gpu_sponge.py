"""Vorticity sponge (Sec. 2.3, sponge term of eq. PNST_org_momentum) on the GPU
against the FP64 oracle, and in ensembles and schedules."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_1506_06513_amd as F
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def _both(n, L, nu, eta, c_sp, thick, body, u0, steps, dtype, mean_mode=F.FLUSI_MEAN_FIXED, **ctl):
    p = O.Params(n, L, nu, eta, mean_mode, c_sp=c_sp, sponge=tuple(thick))
    ins = O.Insect.from_dict(body) if body else None
    ost, oh = O.run(p, u0, steps, O.StepControl(**ctl), ins)
    P = F.Plan(n, L, nu, eta, dtype)
    P.set_sponge(c_sp, thick)
    st = P.new_state(torch.from_numpy(u0))
    h = P.step(st, steps, body, history=True, mean_mode=mean_mode, **ctl).cpu().numpy()
    return O.velocity(p, ost), oh, P.velocity(st).cpu().numpy(), h


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_taylor_green_full_sponge(dtype):
    n, L = 32, 2 * math.pi
    ou, _, u, _ = _both(n, L, 0.02, 1.0, 0.05, (L, 0.0, 0.0), None, W.taylor_green(n), 20, dtype,
                        mean_mode=F.FLUSI_MEAN_FREE, dt_fixed=2e-3)
    assert rel_l2(u, ou) < (1e-11 if dtype == "f64" else 2e-5)
    # the sponge damps: at rate 1/C_sp beyond the viscous decay
    assert np.max(np.abs(ou)) < 0.5 * np.max(np.abs(W.taylor_green(n)))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sphere_with_downstream_sponge_layer(dtype):
    n, L = 48, 4.0
    u0 = W.inflow_noise(n, L, seed=3, rms=1e-2, kmax=6.0)
    ou, oh, u, h = _both(n, L, 0.01, 1e-3, 0.1, (0.5, 0.0, 0.0), W.sphere_body(L), u0, 20, dtype, cfl=0.1)
    assert rel_l2(u, ou) < (1e-11 if dtype == "f64" else 2e-5)
    oF = np.array([d["F"][0] for d in oh])
    assert np.max(np.abs(h[:, 4:7] - oF)) <= (1e-10 if dtype == "f64" else 1e-4) * np.max(np.abs(oF))


def test_insect_with_sponge_on_two_axes():
    n, L = 48, 4.0
    body = W.model_insect(n, L)
    u0 = W.inflow_noise(n, L, seed=4, rms=1e-2, kmax=6.0)
    ou, _, u, _ = _both(n, L, 1 / 136, 5e-4, 0.1, (0.5, 0.75, 0.0), body, u0, 6, "f64", cfl=0.1)
    assert rel_l2(u, ou) < 1e-11


def test_sponge_off_equals_no_sponge_and_schedules_agree():
    n, L = 48, 4.0
    u0 = W.inflow_noise(n, L, seed=5, rms=1e-2, kmax=6.0)
    body = W.sphere_body(L)
    P = F.Plan(n, L, 0.01, 1e-3, "f32")
    a = P.new_state(torch.from_numpy(u0))
    P.step(a, 5, body, cfl=0.1)
    Q = F.Plan(n, L, 0.01, 1e-3, "f32")
    Q.set_sponge(0.1, (0.5, 0.0, 0.0))
    Q.set_sponge(0.0, (0.5, 0.0, 0.0))  # switched off again
    b = Q.new_state(torch.from_numpy(u0))
    Q.step(b, 5, body, cfl=0.1)
    assert torch.equal(P.uhat(a), Q.uhat(b))
    # with the sponge on, every schedule gives the same velocity
    Q.set_sponge(0.1, (0.5, 0.5, 0.0))
    ref = None
    for sc in ({}, {"x_pass": 1, "z_pass": 2, "split_z": 1}, {"x_pass": 2, "y_forward": 2, "z_pass": 1}):
        Q.set_schedule({"y_inverse": 0, "x_pass": 0, "y_forward": 0, "z_pass": 0, "split_z": 0, **sc})
        s = Q.new_state(torch.from_numpy(u0))
        Q.step(s, 5, body, cfl=0.1)
        uh = Q.uhat(s)
        if ref is None:
            ref = uh
        assert torch.equal(uh, ref), sc


def test_mixed_ensemble_with_and_without_sponge():
    L = 4.0
    specs = [(48, (0.5, 0.0, 0.0), W.sphere_body(L)), (48, None, W.model_insect(48, L)),
             (32, (0.0, 0.5, 0.5), W.model_insect(32, L)), (32, None, W.sphere_body(L)),
             (48, (0.25, 0.25, 0.25), None)]
    ens = F.Ensemble("f32")
    pairs = []
    for n, thick, body in specs:
        u0 = W.inflow_noise(n, L, seed=n + (7 if thick else 0), rms=1e-2, kmax=6.0)
        Pa, Pb = F.Plan(n, L, 0.01, 1e-3, "f32"), F.Plan(n, L, 0.01, 1e-3, "f32")
        if thick:
            Pa.set_sponge(0.1, thick)
            Pb.set_sponge(0.1, thick)
        sa, sb = Pa.new_state(torch.from_numpy(u0)), Pb.new_state(torch.from_numpy(u0))
        ens.add(Pa, sa, body, cfl=0.1)
        pairs.append((Pa, sa, Pb, sb, body))
    ens.step(4, graph=True)
    for Pa, sa, Pb, sb, body in pairs:
        Pb.step(sb, 4, body, cfl=0.1)
    torch.cuda.synchronize()
    for i, (Pa, sa, Pb, sb, _) in enumerate(pairs):
        assert torch.equal(Pa.uhat(sa), Pb.uhat(sb)), i
    ens.close()

"""RK4 with explicit diffusion (Sec. 2.4) on the GPU against the FP64 oracle:
Taylor-Green (and the RK4 stability polynomial), an adaptive sphere in inflow
(step cap), a flapping insect (stage-time kinematics), the vorticity sponge,
integrator switches; chunked calls, schedules and the limits of RK4 plans."""
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


def _both(n, L, nu, eta, u0, body, steps, dtype, mean_mode=F.FLUSI_MEAN_FIXED, sponge=None, **ctl):
    p = O.Params(n, L, nu, eta, mean_mode, integrator="rk4",
                 **({} if sponge is None else dict(c_sp=sponge[0], sponge=tuple(sponge[1]))))
    ost, oh = O.run(p, u0, steps, O.StepControl(**ctl), O.Insect.from_dict(body) if body else None)
    P = F.Plan(n, L, nu, eta, dtype)
    P.set_integrator("rk4")
    if sponge is not None:
        P.set_sponge(*sponge)
    st = P.new_state(torch.from_numpy(u0))
    h = P.step(st, steps, body, history=True, mean_mode=mean_mode, **ctl).cpu().numpy()
    return O.velocity(p, ost), oh, P.velocity(st).cpu().numpy(), h, P, st


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_taylor_green_rk4(dtype):
    n, L, nu, dt, steps = 32, 2 * math.pi, 0.05, 0.02, 30
    u0 = W.taylor_green(n)
    ou, _, u, h, _, _ = _both(n, L, nu, 1.0, u0, None, steps, dtype, mean_mode=F.FLUSI_MEAN_FREE, dt_fixed=dt)
    tol = 1e-11 if dtype == "f64" else 2e-5
    assert rel_l2(u, ou) < tol
    z = -2 * nu * dt
    amp = (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24) ** steps
    assert rel_l2(u, amp * u0) < (1e-12 if dtype == "f64" else 2e-6)
    assert np.all(h[:, 1] == dt)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sphere_rk4_adaptive(dtype):
    n, L = 48, 4.0
    u0 = W.inflow_noise(n, L, seed=60, rms=1e-2, kmax=6.0)
    ou, oh, u, h, _, _ = _both(n, L, 0.05, 1e-2, u0, W.sphere_body(L), 12, dtype, cfl=0.2, eta_cap=0.5)
    assert rel_l2(u, ou) < (1e-11 if dtype == "f64" else 2e-5)
    odt = np.array([d["dt"] for d in oh])
    assert np.max(np.abs(h[:, 1] - odt)) <= (1e-13 if dtype == "f64" else 1e-6) * odt.max()
    oF = np.array([d["F"][0] for d in oh])
    assert np.max(np.abs(h[:, 4:7] - oF)) <= (1e-10 if dtype == "f64" else 1e-4) * np.max(np.abs(oF))


def test_viscous_cap_sets_the_step():
    n, L, nu = 32, 2 * math.pi, 0.5
    u0 = W.taylor_green(n)
    ou, oh, u, h, _, _ = _both(n, L, nu, 1.0, u0, None, 4, "f64", mean_mode=F.FLUSI_MEAN_FREE, cfl=5.0)
    K = (n - 1) // 3
    cap = O.RK4_VISC / (nu * 3 * K * K)
    assert np.max(np.abs(h[:, 1] - cap)) < 1e-15 and rel_l2(u, ou) < 1e-11


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_flapping_insect_rk4_uses_stage_times(dtype):
    n, L = 48, 4.0
    u0 = W.inflow_noise(n, L, seed=61, rms=1e-2, kmax=6.0)
    body = W.model_insect(n, L)
    body.update(psi_dot=0.5)
    ou, oh, u, h, _, _ = _both(n, L, 1 / 136, 5e-3, u0, body, 6, dtype, cfl=0.1)
    assert rel_l2(u, ou) < (1e-11 if dtype == "f64" else 2e-5)
    if dtype == "f64":
        for c in range(3):
            oF = np.array([d["F"][c] for d in oh])
            assert np.max(np.abs(h[:, 4 + 6 * c:7 + 6 * c] - oF)) <= 1e-9 * max(1e-12, np.max(np.abs(oF))), c


def test_sponge_with_rk4():
    n, L = 48, 4.0
    u0 = W.inflow_noise(n, L, seed=62, rms=1e-2, kmax=6.0)
    ou, _, u, _, _, _ = _both(n, L, 0.02, 1e-2, u0, W.sphere_body(L), 6, "f64", sponge=(0.1, (0.5, 0.0, 0.0)), cfl=0.1)
    assert rel_l2(u, ou) < 1e-11


def test_integrator_switches_match_oracle():
    """AB2 -> RK4 -> AB2: after RK4 the AB2 history is gone (Euler restart)."""
    n, L, nu, eta = 48, 4.0, 0.02, 1e-2
    u0 = W.inflow_noise(n, L, seed=63, rms=1e-2, kmax=6.0)
    body = W.sphere_body(L)
    ctl = dict(cfl=0.1)
    p = O.Params(n, L, nu, eta, O.MEAN_FIXED)
    st = O.init_state(p, u0)
    ins = O.Insect.from_dict(body)
    P = F.Plan(n, L, nu, eta, "f64")
    s = P.new_state(torch.from_numpy(u0))
    for integ, k in (("ab2", 3), ("rk4", 3), ("ab2", 3)):
        p.integrator = integ
        for _ in range(k):
            st, _ = O.step(p, st, O.StepControl(**ctl), ins)
        P.set_integrator(integ)
        P.step(s, k, body, **ctl)
    assert rel_l2(P.velocity(s).cpu().numpy(), O.velocity(p, st)) < 1e-11


def test_chunks_schedules_and_limits():
    n, L = 48, 4.0
    u0 = W.inflow_noise(n, L, seed=64, rms=1e-2, kmax=6.0)
    body = W.model_insect(n, L)
    P = F.Plan(n, L, 0.01, 5e-3, "f32")
    P.set_integrator("rk4")
    a = P.new_state(torch.from_numpy(u0))
    P.step(a, 4, body, cfl=0.1)
    b = P.new_state(torch.from_numpy(u0))
    P.step(b, 1, body, cfl=0.1)
    P.step(b, 3, body, cfl=0.1)
    assert torch.equal(P.uhat(a), P.uhat(b))
    ref = P.uhat(a)
    for sc in ({"x_pass": 1, "z_pass": 1}, {"x_pass": 2, "y_inverse": 2, "y_forward": 1, "z_pass": 2}):
        P.set_schedule({"y_inverse": 0, "x_pass": 0, "y_forward": 0, "z_pass": 0, "split_z": 0, **sc})
        c = P.new_state(torch.from_numpy(u0))
        P.step(c, 4, body, cfl=0.1)
        assert torch.equal(P.uhat(c), ref), sc
    sched = P.autotune(P.new_state(torch.from_numpy(u0)), body, reps=2, cfl=0.1)
    assert set(sched) >= {"x_pass", "z_pass"}
    ff = dict(W.sphere_body(L), free_flight=True, mass=1.0, inertia=(0.1, 0.1, 0.1))
    with pytest.raises(F.FlusiError) as e:
        P.step(a, 1, ff, cfl=0.1)
    assert e.value.code == F.FLUSI_EUNSUPPORTED
    ens = F.Ensemble("f32")
    with pytest.raises(F.FlusiError) as e:
        ens.add(P, a, ff, cfl=0.1)
    assert e.value.code == F.FLUSI_EUNSUPPORTED
    ens.close()
    assert F.lib().flusi_plan_set_integrator(P.handle, 7) == F.FLUSI_EINVAL


def test_rk4_members_in_ensembles_equal_solo_runs():
    """RK4 and AB2 members of one ensemble (separate groups of the same grid,
    graph replay) equal their solo runs bitwise."""
    specs = [(48, "rk4", W.model_insect(48, 4.0)), (48, "ab2", W.model_insect(48, 4.0)),
             (32, "rk4", W.sphere_body(4.0)), (48, "rk4", None)]
    ens = F.Ensemble("f32")
    pairs = []
    for k, (n, integ, body) in enumerate(specs):
        u0 = W.inflow_noise(n, 4.0, seed=70 + k, rms=1e-2, kmax=6.0)
        Pa, Pb = F.Plan(n, 4.0, 0.01, 5e-3, "f32"), F.Plan(n, 4.0, 0.01, 5e-3, "f32")
        Pa.set_integrator(integ)
        Pb.set_integrator(integ)
        sa, sb = Pa.new_state(torch.from_numpy(u0)), Pb.new_state(torch.from_numpy(u0))
        ens.add(Pa, sa, body, cfl=0.1)
        pairs.append((Pa, sa, Pb, sb, body))
    assert ens.size() == (4, 3)
    ens.step(3, graph=True)
    ens.step(2)
    for Pa, sa, Pb, sb, body in pairs:
        Pb.step(sb, 5, body, cfl=0.1)
    torch.cuda.synchronize()
    for i, (Pa, sa, Pb, sb, _) in enumerate(pairs):
        assert torch.equal(Pa.uhat(sa), Pb.uhat(sb)), i
    ens.close()

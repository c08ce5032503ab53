"""Tile-variant schedules and the autotuner (needs an MI355X).

Every schedule performs the same operations per value, so the velocity must
be bitwise independent of it; only the order of the FP64 diagnostic sums may
change (x-pass variant)."""
import pytest
import torch

import paper_1506_06513_amd as F
import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("y_inverse", "x_pass", "y_forward", "z_pass", "split_z")


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


def _case(n, body):
    L = 4.0
    if body == "insect":
        return L, W.model_insect(n, L), W.inflow_noise(n, L, seed=2, rms=1e-2, kmax=6.0)
    return L, W.sphere_body(L), W.inflow_noise(n, L, seed=3, rms=1e-2, kmax=6.0)


SCHEDULES = [dict(zip(KEYS, v)) for v in
             ((1, 1, 1, 1, 0), (1, 1, 1, 1, 1), (0, 1, 0, 1, 0), (1, 0, 1, 0, 1), (0, 0, 0, 0, 1),
              (2, 2, 2, 2, 0), (2, 0, 1, 2, 1), (0, 2, 2, 1, 0))]


@pytest.mark.parametrize("n,body,dtype", [(24, "insect", "f64"), (48, "sphere", "f32"), (96, "insect", "f32"),
                                          (192, "insect", "f32"), (128, "sphere", "f64")])
def test_velocity_is_independent_of_the_schedule(n, body, dtype):
    L, ins, u0 = _case(n, body)
    P = F.Plan(n, L, 1 / 136, 5e-4, dtype)
    ref = P.new_state(torch.from_numpy(u0))
    h0 = P.step(ref, 4, ins, cfl=0.1, history=True)
    for sc in SCHEDULES:
        P.set_schedule(sc)
        assert P.schedule() == sc
        st = P.new_state(torch.from_numpy(u0))
        h = P.step(st, 4, ins, cfl=0.1, history=True)
        torch.cuda.synchronize()
        assert torch.equal(P.uhat(st), P.uhat(ref)), sc
        assert P.time(st) == P.time(ref)
        # t, dt and max|u| exactly; energy, force and torque sums to round-off
        assert torch.equal(h[:, :3], h0[:, :3]), sc
        scale = h0[:, 3:].abs().max()
        assert (h[:, 3:] - h0[:, 3:]).abs().max() <= 1e-12 * scale, sc


def test_bad_schedule_is_rejected():
    P = F.Plan(32, 4.0, 0.01, 1e-3, "f32")
    with pytest.raises(F.FlusiError) as e:
        P.set_schedule({"x_pass": 3})
    assert e.value.code == F.FLUSI_EINVAL


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_autotune_leaves_the_state_and_sets_a_schedule(dtype):
    n = 64
    L, ins, u0 = _case(n, "insect")
    P = F.Plan(n, L, 1 / 136, 5e-4, dtype)
    st = P.new_state(torch.from_numpy(u0))
    P.step(st, 2, ins, cfl=0.1)
    before = st.clone()
    sc = P.autotune(st, ins, reps=4, cfl=0.1)
    torch.cuda.synchronize()
    assert torch.equal(st, before)
    assert set(sc) == set(KEYS) and all(v in (0, 1, 2) for v in sc.values()) and sc["split_z"] in (0, 1)
    assert P.schedule() == sc
    # stepping with the tuned schedule matches the default schedule
    Q = F.Plan(n, L, 1 / 136, 5e-4, dtype)
    s2 = Q.new_state(torch.from_numpy(u0))
    Q.step(s2, 2, ins, cfl=0.1)
    P.step(st, 3, ins, cfl=0.1)
    Q.step(s2, 3, ins, cfl=0.1)
    assert torch.equal(P.uhat(st), Q.uhat(s2))


def test_ensemble_autotune_keeps_member_results():
    specs = [(32, "sphere"), (48, "insect"), (48, "sphere"), (64, "insect")]
    ens = F.Ensemble("f32")
    members, solos = [], []
    for n, body in specs:
        L, ins, u0 = _case(n, body)
        P = F.Plan(n, L, 1 / 150, 4e-4, "f32")
        st = P.new_state(torch.from_numpy(u0))
        ens.add(P, st, ins, cfl=0.1)
        members.append((P, st))
        Q = F.Plan(n, L, 1 / 150, 4e-4, "f32")
        solos.append((Q, Q.new_state(torch.from_numpy(u0)), ins))
    before = [s.clone() for _, s in members]
    ens.autotune(reps=3)
    torch.cuda.synchronize()
    for (P, st), b in zip(members, before):
        assert torch.equal(st, b)
    ens.step(4, graph=True)
    for Q, s, ins in solos:
        Q.step(s, 4, ins, cfl=0.1)
    torch.cuda.synchronize()
    for (P, st), (Q, s, _) in zip(members, solos):
        assert torch.equal(P.uhat(st), Q.uhat(s))
    ens.close()

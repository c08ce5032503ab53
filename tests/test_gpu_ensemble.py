"""Batched stepping of many simulations (flusi_ensemble_*) on the GPU.

Each member of an ensemble follows the arithmetic of a solo flusi_step on its
own plan, so results must match solo runs bit for bit; graph replays must
match eager calls bit for bit; and members are checked against the FP64
oracle (Algorithm 1) like solo runs."""
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


def _members():
    """Mixed sizes, bodies and parameters (radix-3 size 48 included)."""
    L = 4.0
    out = []
    out.append(dict(n=32, L=2 * math.pi, nu=0.01, eta=1.0, body=None, u0=W.taylor_green(32),
                    ctl=dict(cfl=0.3, mean_mode=F.FLUSI_MEAN_FREE)))
    out.append(dict(n=48, L=L, nu=0.02, eta=1e-3, body=W.sphere_body(L),
                    u0=W.inflow_noise(48, L, seed=5, rms=1e-2, kmax=6.0), ctl=dict(cfl=0.1)))
    out.append(dict(n=48, L=L, nu=1 / 136, eta=5e-4, body=W.model_insect(48, L),
                    u0=np.zeros((3, 48, 48, 48)), ctl=dict(cfl=0.1)))
    out.append(dict(n=64, L=L, nu=1 / 200, eta=2.5e-4, body=W.model_insect(64, L, phi_m=math.radians(60)),
                    u0=W.inflow_noise(64, L, seed=6, rms=1e-2, kmax=6.0), ctl=dict(cfl=0.1)))
    out.append(dict(n=32, L=L, nu=0.05, eta=1e-3, body=W.sphere_body(L),
                    u0=W.inflow_noise(32, L, seed=7, rms=1e-2, kmax=6.0), ctl=dict(cfl=0.1)))
    return out


def _setup(spec, dtype):
    P = F.Plan(spec["n"], spec["L"], spec["nu"], spec["eta"], dtype)
    st = P.new_state(torch.from_numpy(spec["u0"]))
    return P, st


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_members_equal_solo_runs_bitwise(dtype):
    specs = _members()
    ens = F.Ensemble(dtype)
    members, solos = [], []
    for sp in specs:
        P, st = _setup(sp, dtype)
        h = torch.zeros((5, F.FLUSI_NDIAG), dtype=torch.float64, device=st.device)
        ens.add(P, st, sp["body"], history=h, **sp["ctl"])
        members.append((P, st, h))
        solos.append(_setup(sp, dtype))
    assert ens.size() == (5, 3)
    for call in range(2):
        ens.step(5)
        for sp, (Ps, ss) in zip(specs, solos):
            hs = Ps.step(ss, 5, sp["body"], history=True, **sp["ctl"])
            sp["hs"] = hs
        torch.cuda.synchronize()
        for sp, (P, st, h), (Ps, ss) in zip(specs, members, solos):
            assert torch.equal(P.uhat(st), Ps.uhat(ss)), (sp["n"], call)
            assert P.time(st) == Ps.time(ss)
            assert torch.equal(h, sp["hs"])
    ens.close()


def test_graph_replays_equal_eager_calls():
    specs = _members()
    eager, graph = F.Ensemble("f32"), F.Ensemble("f32")
    a, b = [], []
    for sp in specs:
        Pa, sa = _setup(sp, "f32")
        Pb, sb = _setup(sp, "f32")
        eager.add(Pa, sa, sp["body"], **sp["ctl"])
        graph.add(Pb, sb, sp["body"], **sp["ctl"])
        a.append((Pa, sa))
        b.append((Pb, sb))
    for call in range(4):
        eager.step(3)
        graph.step(3, graph=True)
        # eager work of the program between replays
        vel = [P.velocity(s) for P, s in b]
        torch.cuda.synchronize()
        for (Pa, sa), (Pb, sb), v in zip(a, b, vel):
            assert torch.equal(Pa.uhat(sa), Pb.uhat(sb)), call
            assert torch.isfinite(v).all()
    eager.close()
    graph.close()


def test_four_members_match_the_oracle_for_20_steps():
    specs = [s for s in _members() if s["n"] <= 48][:4]
    ens = F.Ensemble("f32")
    members = []
    for sp in specs:
        P, st = _setup(sp, "f32")
        ens.add(P, st, sp["body"], **sp["ctl"])
        members.append((P, st))
    ens.step(20, graph=True)
    torch.cuda.synchronize()
    for sp, (P, st) in zip(specs, members):
        ctl = sp["ctl"]
        p = O.Params(sp["n"], sp["L"], sp["nu"], sp["eta"], ctl.get("mean_mode", O.MEAN_FIXED))
        ins = O.Insect.from_dict(sp["body"]) if sp["body"] else None
        ost, _ = O.run(p, sp["u0"], 20, O.StepControl(cfl=ctl["cfl"]), ins)
        assert rel_l2(P.velocity(st).cpu().numpy(), O.velocity(p, ost)) < 2e-5, sp["n"]


def test_removed_member_stops_and_others_continue():
    specs = _members()[:3]
    ens = F.Ensemble("f64")
    members = []
    ids = []
    for sp in specs:
        P, st = _setup(sp, "f64")
        ids.append(ens.add(P, st, sp["body"], **sp["ctl"]))
        members.append((P, st))
    ens.step(2, graph=True)
    ens.remove(ids[1])
    assert ens.size() == (2, 2)
    frozen = members[1][0].uhat(members[1][1]).clone()
    t_before = [P.time(s)[1] for P, s in members]
    ens.step(2, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(frozen, members[1][0].uhat(members[1][1]))
    t_after = [P.time(s)[1] for P, s in members]
    assert t_after == [t_before[0] + 2, t_before[1], t_before[2] + 2]
    # a re-added member continues from its state
    ens.add(members[1][0], members[1][1], specs[1]["body"], **specs[1]["ctl"])
    ens.step(1)
    torch.cuda.synchronize()
    assert members[1][0].time(members[1][1])[1] == t_before[1] + 1
    ens.close()


@pytest.mark.parametrize("graph", [False, True])
def test_member_plan_option_change_rebuilds_the_tables(graph):
    """Switching a member plan's sponge on (which replaces its scratch buffer)
    and changing its schedule after it joined: the next ensemble call rebuilds
    the launch tables (and drops captured graphs), so the member still equals
    flusi_step on its plan with the new options, bit for bit."""
    specs = _members()[1:4]
    ens = F.Ensemble("f64")
    members, solos = [], []
    for sp in specs:
        P, st = _setup(sp, "f64")
        ens.add(P, st, sp["body"], **sp["ctl"])
        members.append((P, st))
        solos.append(_setup(sp, "f64"))
    ens.step(2, graph=graph)
    for sp, (Ps, ss) in zip(specs, solos):
        Ps.step(ss, 2, sp["body"], **sp["ctl"])
    torch.cuda.synchronize()
    # sponge on member 0 (new scratch buffer), another z-pass form on member 2
    members[0][0].set_sponge(0.1, (0.5, 0.0, 0.0))
    solos[0][0].set_sponge(0.1, (0.5, 0.0, 0.0))
    members[2][0].set_schedule(dict(z_pass=1, split_z=1))
    solos[2][0].set_schedule(dict(z_pass=1, split_z=1))
    for call in range(2):
        ens.step(3, graph=graph)
        for sp, (Ps, ss) in zip(specs, solos):
            Ps.step(ss, 3, sp["body"], **sp["ctl"])
        torch.cuda.synchronize()
        for sp, (P, st), (Ps, ss) in zip(specs, members, solos):
            assert torch.equal(P.uhat(st), Ps.uhat(ss)), (sp["n"], call)
            assert P.time(st) == Ps.time(ss)
    ens.close()

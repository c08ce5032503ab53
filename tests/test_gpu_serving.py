"""Request loop with continuous batching (flusi_server_*) on the GPU.

Requests of different grids, Re, C_eta and bodies arrive while others run;
each result must equal the same request stepped alone (bitwise: the server
runs every request through the same kernels as flusi_step, and splitting a
run into chunks does not change it)."""
import math
import time

import numpy as np
import pytest
import torch

import paper_1506_06513_amd as F
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


def _requests():
    L = 4.0
    return [
        # long-running first request: the others arrive while it is on the device
        dict(n=128, L=L, nu=0.01, eta=1e-3, steps=300, insect=W.sphere_body(L),
             u0=W.inflow_noise(128, L, seed=10, rms=1e-3, kmax=8.0), ctl=dict(cfl=0.1)),
        dict(n=32, L=L, nu=0.02, eta=1e-3, steps=12, insect=W.sphere_body(L),
             u0=W.inflow_noise(32, L, seed=11, rms=1e-2, kmax=6.0), ctl=dict(cfl=0.1)),
        dict(n=48, L=L, nu=1 / 120, eta=5e-4, steps=20, insect=W.model_insect(48, L), u0=None, ctl=dict(cfl=0.1)),
        dict(n=64, L=L, nu=1 / 300, eta=3e-4, steps=8, insect=W.model_insect(64, L, phi_m=math.radians(55)),
             u0=None, ctl=dict(cfl=0.1)),
        dict(n=32, L=2 * math.pi, nu=0.01, eta=1.0, steps=15, insect=None, u0=W.taylor_green(32),
             ctl=dict(cfl=0.3, mean_mode=F.FLUSI_MEAN_FREE)),
        dict(n=48, L=L, nu=0.01, eta=1e-3, steps=25, insect=W.sphere_body(L),
             u0=W.inflow_noise(48, L, seed=12, rms=1e-2, kmax=6.0), ctl=dict(cfl=0.1)),
        dict(n=24, L=L, nu=0.02, eta=1e-3, steps=7, insect=W.sphere_body(L),
             u0=W.inflow_noise(24, L, seed=13, rms=1e-2, kmax=4.0), ctl=dict(cfl=0.1)),
    ]


def _alone(rq, dtype):
    P = F.Plan(rq["n"], rq["L"], rq["nu"], rq["eta"], dtype)
    u0 = rq["u0"] if rq["u0"] is not None else np.zeros((3, rq["n"], rq["n"], rq["n"]))
    st = P.new_state(torch.from_numpy(u0))
    P.step(st, rq["steps"], rq["insect"], **rq["ctl"])
    rc, diag = P.forces(st)
    return P.velocity(st).cpu().numpy(), diag


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_each_result_is_the_same_alone_and_in_the_mix(dtype):
    reqs = _requests()
    srv = F.Server(dtype, hbm_budget=8 << 30, max_chunk=4)
    ids = []
    for rq in reqs:
        ids.append(srv.submit(rq["n"], rq["L"], rq["nu"], rq["eta"], rq["steps"], rq["insect"], rq["u0"], **rq["ctl"]))
        time.sleep(0.002)  # staggered arrivals: later requests join running ones
    out = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_active"] >= 2  # requests really overlapped on the device
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    for rq, (rc, u, diag, lat) in zip(reqs, out):
        assert rc == 0 and lat > 0
        ua, da = _alone(rq, dtype)
        assert np.array_equal(u, ua), rq["n"]
        assert np.array_equal(diag, da), rq["n"]


def test_admission_keeps_within_the_budget():
    n = 48
    per = F.flusi_request_bytes(n, F.FLUSI_F32)
    srv = F.Server("f32", hbm_budget=int(2.5 * per), max_chunk=5)
    L = 4.0
    ids = [srv.submit(n, L, 0.01 + 0.002 * k, 1e-3, 10, W.sphere_body(L), None, cfl=0.1) for k in range(5)]
    res = [srv.wait(i, want_u=False) for i in ids]
    st = srv.stats()
    srv.close()
    assert all(r[0] == 0 for r in res)
    assert st["completed"] == 5 and st["peak_active"] <= 2 and st["peak_bytes"] <= int(2.5 * per)
    # the footprint covers what a plan and a state allocate
    ws, sb = F.flusi_sizes(n, F.FLUSI_F32)
    P = F.Plan(n, L, 0.01, 1e-3, "f32")
    assert F.flusi_plan_workspace_bytes(P.handle) == ws and F.flusi_state_bytes(P.handle) == sb
    assert per > ws + sb


def test_oversized_request_is_rejected_and_bad_state_reported():
    srv = F.Server("f32", hbm_budget=F.flusi_request_bytes(48, F.FLUSI_F32), max_chunk=3)
    with pytest.raises(F.FlusiError) as e:
        srv.submit(64, 4.0, 0.01, 1e-3, 5, None, None, cfl=0.1)
    assert e.value.code == F.FLUSI_ENOMEM
    u0 = W.inflow_noise(32, 4.0, seed=0, rms=1e-3, kmax=6.0)
    u0[0, 1, 2, 3] = np.nan
    bad = srv.submit(32, 4.0, 0.01, 1e-3, 6, W.sphere_body(4.0), u0, cfl=0.1)
    good = srv.submit(32, 4.0, 0.01, 1e-3, 6, W.sphere_body(4.0), np.nan_to_num(u0), cfl=0.1)
    rb = srv.wait(bad, want_u=False)
    rg = srv.wait(good, want_u=False)
    srv.close()
    assert rb[0] == F.FLUSI_ENONFINITE
    assert rg[0] == 0

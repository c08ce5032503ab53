"""Benchmark of the pseudo-spectral penalized Navier-Stokes step on one MI355X.

Workload (default, the largest single-GPU configuration): 256^3 periodic box
L = 4 with the model insect (ellipsoid body, two flat elliptic wings flapping
at f = 1 with stroke +-70 deg and feathering +-45 deg), mask and solid
velocity rebuilt every step, nu = 1/136, C_eta = 2.5e-4, adaptive dt at CFL
0.1 (capped at C_eta/2), fluid at rest.  One step = one pass of the whole hot
path: kinematics, mask on the fly, u x w and penalization, 2/3 rule,
projection, IF-AB2 update, FP64 max|u| / force / energy reductions and the
adaptive dt.

Prints one JSON line.  `value` is FP32 Mpoint-steps/s (points x steps / s);
the FP64 figure, each precision's error against the FP64 oracle, the roofline
of the dominant kernel (live HIP-event timing over a timed region, algorithmic
bytes from the pruned byte model) and the oracle's CPU throughput on a bounded
sample are reported beside it.  Schedules are autotuned before the timed
region (--no-autotune: defaults).  The default run adds sub-objects:
`sphere128` (128^3 sphere in inflow, FP32 and FP64 with their roofline),
`ensemble48` (48 seeded insect simulations on mixed grids advanced by batched
launches replayed from a hipGraph, against the same members stepped one by
one), `serving` (a Poisson-arrival request stream with a 512^3 insect: p50/p99
latency and throughput, and a saturated stream for capacity), plus `sponge`,
`freeflight`, `rk4` and `box192` (the sphere workload with a vorticity sponge
layer, with the sphere in free flight, stepped with RK4, and in the 6x4x4 box
at 192x128x128 points).  --workload selects sphere128, freefall128, tg32,
box192, ensemble48 or serve as the main line instead.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpoint-steps/s (AB2 RHS) FP32 vs FP64 at stated err; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def x_rows(nx: int, cbytes: int, variant: int = 0) -> int:
    """Rows per x-pass workgroup (the kernels' rows_x): 3*rows*nx ~ 3072 complex
    values, halved per variant, at least 2, except one row where two rows of
    nine columns would pass 150 KiB of LDS, or for the smaller variants of rows
    of 1024 points or more."""
    c, p = 1024 // nx, 2
    while p * 2 <= c:
        p *= 2
    p >>= variant
    if p < 2:
        p = 1 if (variant > 0 and nx >= 1024) else 2
    if p == 2 and 9 * (nx + nx // 16 + 1) * cbytes > 150 * 1024:
        p = 1
    return p


def pass_bytes(n: int, cbytes: int, split_z: bool, x_variant: int = 0, nx: int | None = None) -> dict:
    """Algorithmic HBM bytes per launch of each pass of the pruned schedule on
    an nx x n x n grid (nx = n by default).

    K = (n-1)//3, KP = (nx-1)//3 + 1 kept kx, M = 2K+1 kept ky and kz, Q = M*KP.
    z-partials [6][n][Q], y-partials [6][n][n][KP], x-output [3][n][n][KP],
    y-output [3][n][Q], state u_hat and previous right-hand side [3][M][Q] each.
    z_pass is forward z + projection + AB2 (+ curl and inverse z when fused);
    z_inverse is curl + inverse z from the state."""
    nx = n if nx is None else nx
    K = (n - 1) // 3
    KP, M = (nx - 1) // 3 + 1, 2 * K + 1
    Q = M * KP
    s = cbytes
    nwg = n * n // x_rows(nx, cbytes, x_variant)
    zup = (3 * n * Q + 4 * 3 * M * Q) * s
    return {
        "z_inverse": (3 * M * Q + 6 * n * Q) * s,
        "y_inverse": (6 * n * Q + 6 * n * n * KP) * s,
        "x_pass": (6 * n * n * KP + 3 * n * n * KP) * s + nwg * 39 * 8,
        "y_forward": (3 * n * n * KP + 3 * n * Q) * s + nwg * 39 * 8,
        "z_pass": zup if split_z else zup + 6 * n * Q * s,
    }


def step_bytes(n: int, cbytes: int, nx: int | None = None) -> int:
    """Bytes the fused four-pass schedule must move per step (the algorithmic
    model; a split z-pass re-reads u_hat, which is not counted)."""
    b = pass_bytes(n, cbytes, split_z=False, nx=nx)
    return b["y_inverse"] + b["x_pass"] + b["y_forward"] + b["z_pass"]


def source_hash() -> str:
    """Hash of the HIP sources; counter summaries are valid only for this hash."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1506_06513_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(workload: str, kernel_prefix: str):
    """HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE) of a kernel from
    the committed rocprofv3 summary, or None when the summary is missing or
    was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{workload}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read().splitlines()
    if f"csrc_sha256: {source_hash()}" not in txt:
        return None
    for line in txt:
        if line.startswith("traffic ") and line[len("traffic "):].startswith(kernel_prefix):
            f, w = line.split()[-2:]
            return int(f) + int(w)
    return None


def moving_body(ins) -> bool:
    """Whether a body's kinematics change with time (evaluated every step)."""
    return bool(ins) and bool(ins.get("wings") or ins.get("free_flight") or ins.get("psi_dot")
                               or ins.get("beta_dot") or ins.get("gamma_dot"))


def kernel_of_pass(pass_name: str, n: int, real: str, sched: dict, nc: int, dyn: bool, nx: int | None = None) -> str:
    """Kernel name (as rocprofv3 prints it) of a pass under a schedule on an
    nx x n x n grid (nx = n: cubic)."""
    split = sched["split_z"]
    g = f"{n if nx is None else nx}, {n}"
    return {
        "z_pass": f"k_zpass<{real}, {g}, {2 if split else 1}, {sched['z_pass']}, false>",
        "z_inverse": f"k_zpass<{real}, {g}, 3, {sched['z_pass']}, false>",
        "x_pass": f"k_xpass<{real}, {g}, {nc}, {sched['x_pass']}, false>",
        "y_inverse": f"k_ypass<{real}, {g}, 1, {2 if dyn else 0}, {sched['y_inverse']}>",
        "y_forward": f"k_ypass<{real}, {g}, -1, 1, {sched['y_forward']}>",
    }[pass_name]


def note(msg: str):
    """Progress line on stderr (the JSON result line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_workload(name: str):
    import workloads as W
    if name == "sphere128":
        wl = W.WORKLOADS["sphere128"]
        n, L = wl["n"], wl["L"]
        u0 = W.inflow_noise(n, L, seed=wl["seed"], rms=1e-3, kmax=8.0)
        body = W.sphere_body(L)
        desc = ("128^3 box L=4, sphere R=0.5 tanh mask 2dx, inflow (1,0,0) + solenoidal noise rms 1e-3 "
                "|k|<=8 (seed 0), nu=0.01, C_eta=1e-3, adaptive dt CFL 0.1 capped at C_eta/2")
        return dict(n=n, L=L, nu=wl["nu"], eta=wl["eta"], u0=u0, insect=body, cfl=0.1, dt_fixed=0.0,
                    desc=desc, default_steps=wl["steps"])
    if name == "box192":
        wl = W.WORKLOADS["sphere128"]
        n, nx, L = 128, 192, wl["L"]
        u0 = W.inflow_noise(n, L, seed=wl["seed"], rms=1e-3, kmax=8.0, nx=nx)
        body = dict(W.sphere_body(L), x_cntr=(2.4, 2.0, 2.0))
        desc = ("192x128x128 box 6x4x4 (one spacing 1/32, the paper's box shape), sphere R=0.5 at (2.4, 2, 2) "
                "tanh mask 2dx, inflow (1,0,0) + solenoidal noise rms 1e-3 |k|<=8 (seed 0), nu=0.01, "
                "C_eta=1e-3, adaptive dt CFL 0.1 capped at C_eta/2")
        return dict(n=n, nx=nx, L=L, nu=wl["nu"], eta=wl["eta"], u0=u0, insect=body, cfl=0.1, dt_fixed=0.0,
                    desc=desc, default_steps=wl["steps"])
    if name == "box1152":
        # the paper's box (Sec. 4 and 6): 6x4x4 at 1152x768x768 points, one
        # spacing 1/192; the model insect at (2.4, 2, 2) in a fluid at rest
        n, nx, L = 768, 1152, 4.0
        wl = W.WORKLOADS["insect256"]
        body = dict(W.model_insect(n, L), x_cntr=(2.4, 2.0, 2.0))
        desc = ("1152x768x768 box 6x4x4 (the paper's box and resolution, one spacing 1/192), model insect at "
                "(2.4, 2, 2) (ellipsoid body + two flapping elliptic wings), nu=1/136, C_eta=2.5e-4, CFL 0.1, "
                "fluid at rest")
        return dict(n=n, nx=nx, L=L, nu=wl["nu"], eta=wl["eta"], u0=None, insect=body, cfl=0.1, dt_fixed=0.0,
                    desc=desc, default_steps=10)
    if name == "freefall128":
        wl = build_workload("sphere128")
        wl["insect"] = W.free_sphere(wl["insect"])
        wl["desc"] = wl["desc"] + "; the sphere in free flight (density 2, g = 1 along -z, 6 DoF)"
        return wl
    if name == "insect256":
        wl = W.WORKLOADS["insect256"]
        n, L = wl["n"], wl["L"]
        u0 = np.zeros((3, n, n, n))
        body = W.model_insect(n, L)
        desc = ("256^3 box L=4, ellipsoid body + two elliptic flapping wings (stroke +-70 deg, feathering "
                "+-45 deg, f=1), mask rebuilt every step, nu=1/136, C_eta=2.5e-4, CFL 0.1, fluid at rest")
        return dict(n=n, L=L, nu=wl["nu"], eta=wl["eta"], u0=u0, insect=body, cfl=0.1, dt_fixed=0.0,
                    desc=desc, default_steps=200)
    if name == "tg32":
        wl = W.WORKLOADS["tg32"]
        n = wl["n"]
        return dict(n=n, L=wl["L"], nu=wl["nu"], eta=wl["eta"], u0=W.taylor_green(n), insect=None, cfl=0.0,
                    dt_fixed=wl["dt_fixed"], desc="32^3 Taylor-Green, nu=0.01, dt=1e-3", default_steps=100)
    raise SystemExit(f"unknown workload {name}")


# --schedule-file: schedules chosen by the first run are stored and reused by
# later runs (profiler passes then see the same kernels as the timed run)
SCHED_PIN = {"path": None, "data": {}}


def pinned_schedule(key, apply, choose):
    """The schedule stored under key (applied with apply), else choose() and store it."""
    d = SCHED_PIN["data"]
    if SCHED_PIN["path"] and key in d:
        apply(d[key])
        return d[key]
    s = choose()
    if SCHED_PIN["path"]:
        d[key] = s
        with open(SCHED_PIN["path"], "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
    return s


def gpu_run(F, torch, wl, dtype, steps, warmup, tune=True, sponge=None, integrator="ab2"):
    P = F.Plan(wl["n"], wl["L"], wl["nu"], wl["eta"], dtype, nx=wl.get("nx"))
    if sponge:
        P.set_sponge(*sponge)
    P.set_integrator(integrator)
    kw = dict(dt_fixed=wl["dt_fixed"], cfl=wl["cfl"], eta_cap=0.5, mean_mode=F.FLUSI_MEAN_FIXED)
    if wl["u0"] is None:  # fluid at rest, built on the device
        u0 = torch.zeros((3,) + P.shape, dtype=P.rdt, device="cuda")
    else:
        u0 = torch.from_numpy(wl["u0"])
    st = P.new_state(u0)
    if warmup:
        P.step(st, warmup, wl["insect"], **kw)
    ins = wl["insect"] or {}
    key = (f"{wl.get('nx') or wl['n']}x{wl['n']}|{dtype}|{integrator}|sponge{int(bool(sponge))}|"
           f"wings{int(bool(ins.get('wings')))}|body{int(bool(ins))}|ff{int(bool(ins.get('free_flight')))}")
    sched = pinned_schedule(key, P.set_schedule,
                            lambda: P.autotune(st, wl["insect"], reps=10, **kw) if tune else P.schedule())
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    P.step(st, steps, wl["insect"], **kw)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    rc, diag = P.forces(st)
    if rc != 0:
        raise SystemExit(f"state stopped with status {rc}")
    # second timed region with per-pass events (dominant-kernel roofline)
    F.flusi_profile(P.handle, True)
    P.step(st, steps, wl["insect"], **kw)
    ms, cnt = F.flusi_pass_times(P.handle)
    F.flusi_profile(P.handle, False)
    torch.cuda.synchronize()
    return dict(wall_s=wall, ev_ms=ev_ms, pass_ms=ms, pass_cnt=cnt, diag=diag, schedule=sched)


def ensemble_run(F, torch, count=48, steps=200, chunk=20, seed=1, tune=True):
    """Batched ensemble (seeded insects on mixed grids, FP32): one graph of
    `chunk` steps for all members, replayed steps/chunk times in the timed
    region; then the same members stepped one by one for comparison."""
    import workloads as W
    specs = W.ensemble_members(count, seed=seed)
    ens = F.Ensemble("f32")
    members = []
    for sp in specs:
        P = F.Plan(sp["n"], sp["L"], sp["nu"], sp["eta"], "f32")
        st = P.new_state(torch.zeros((3, sp["n"], sp["n"], sp["n"]), dtype=torch.float32, device="cuda"))
        ens.add(P, st, sp["insect"], cfl=0.1)
        members.append((P, st, sp))
    nmem, ngroups = ens.size()
    keys = sorted({f"ensemble|{sp['n']}" for sp in specs})
    if SCHED_PIN["path"] and all(k in SCHED_PIN["data"] for k in keys):
        for P, st, sp in members:
            P.set_schedule(SCHED_PIN["data"][f"ensemble|{sp['n']}"])
    elif tune:
        ens.autotune(reps=5)
    scheds = {}
    for P, st, sp in members:
        scheds.setdefault(str(sp["n"]), P.schedule())
    for n, sc in scheds.items():
        pinned_schedule(f"ensemble|{n}", lambda s_: None, lambda: sc)
    ens.step(chunk, graph=True)  # capture + warm-up
    torch.cuda.synchronize()
    pts = sum(float(sp["n"]) ** 3 for sp in specs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps // chunk):
        ens.step(chunk, graph=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    done = steps // chunk * chunk
    for P, st, sp in members:
        rc, _ = P.forces(st)
        if rc != 0:
            raise SystemExit(f"ensemble member {sp['id']} stopped with status {rc}")
    ens.close()
    # the same members, one flusi_step call each, for `chunk` steps
    e0.record()
    for P, st, sp in members:
        P.step(st, chunk, sp["insect"], cfl=0.1)
    e1.record()
    torch.cuda.synchronize()
    ms_solo = e0.elapsed_time(e1)
    grids = {}
    for sp in specs:
        grids[sp["n"]] = grids.get(sp["n"], 0) + 1
    v = pts * done / (ms / 1e3) / 1e6
    v_solo = pts * chunk / (ms_solo / 1e3) / 1e6
    return {"value": round(v, 2), "unit": "Mpoint-steps/s", "members": nmem, "size_groups": ngroups,
            "grids": {str(k): c for k, c in sorted(grids.items())}, "steps": done, "graph_chunk": chunk,
            "ms": round(ms, 3), "point_steps": pts * done, "dtype": "f32",
            "one_by_one": {"value": round(v_solo, 2), "steps": chunk, "ms": round(ms_solo, 3)},
            "batching_speedup": round(v / v_solo, 3),
            "schedules": scheds if tune else "default",
            "description": f"{count} seeded insects (grids {{64,96,128,192}}, Re 50-500, C_eta 1e-4..1e-3, "
                           f"stroke 50-80 deg; seed {seed}), fluid at rest, CFL 0.1"}


def serve_run(F, torch, count=120, seed=2, budget_gib=32.0, chunk=20, big_n=512, big_steps=2000, saturate=False):
    """Serving stream: requests submitted at their Poisson arrival times to a
    flusi server (FP32, HBM budget budget_gib); latency from submit to result.
    saturate=True submits every request at once (offered load above capacity):
    its throughput is the serving capacity."""
    import workloads as W
    reqs = W.serve_stream(count, seed=seed, big_n=big_n, big_steps=big_steps)
    if saturate:
        reqs = [dict(r, arrival=0.0) for r in reqs]
    big = [r for r in reqs if r["turbulent"]][0]
    t_ic = time.perf_counter()
    big_u0 = W.turbulent_inflow(big["n"], big["L"], seed=big["seed"], intensity=0.1, kmax=32.0).astype(np.float32)
    t_ic = time.perf_counter() - t_ic
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(free * 0.8, budget_gib * (1 << 30)))
    srv = F.Server("f32", hbm_budget=budget, max_chunk=chunk)
    ids = []
    t0 = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t0
        if r["arrival"] > now:
            time.sleep(r["arrival"] - now)
        ids.append(srv.submit(r["n"], r["L"], r["nu"], r["eta"], r["steps"], r["insect"],
                              big_u0 if r["turbulent"] else None, cfl=0.1))
    res = [srv.wait(i, want_u=False) for i in ids]
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    bad = [r["id"] for r, x in zip(reqs, res) if x[0] != 0]
    if bad:
        raise SystemExit(f"serving: requests {bad} failed")
    grids = {}
    for r in reqs:
        grids[r["n"]] = grids.get(r["n"], 0) + 1
    return {"p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2), "max_ms": round(st["max_ms"], 2),
            "value": round(st["mpoint_steps_per_s"], 2), "unit": "Mpoint-steps/s",
            "requests": count, "completed": st["completed"], "grids": {str(k): v for k, v in sorted(grids.items())},
            "large_request_latency_ms": round(res[big["id"]][3], 2),
            "peak_active": st["peak_active"], "peak_bytes": st["peak_bytes"], "hbm_budget_bytes": budget,
            "max_chunk": chunk, "arrival_span_s": round(reqs[-1]["arrival"], 2), "wall_s": round(wall, 2),
            "busy_s": round(st["busy_s"], 2), "point_steps": st["point_steps"], "dtype": "f32",
            "initial_field_s": round(t_ic, 1),
            "arrivals": "all at t = 0 (saturated)" if saturate else "Poisson, mean 4/s",
            "description": f"{count} requests, Poisson arrivals mean 4/s (seed {seed}): one {big['n']}^3 insect "
                           f"in k^-5/3 turbulent inflow (intensity 0.1, |k| 1-32, {big['steps']} steps), the rest "
                           f"insects on {{64,96,128,192}}^3 (Re 50-500, C_eta 1e-4..1e-3, 200 steps, at rest); "
                           f"FP32 with FP64 reductions; admitted by footprint within the HBM budget"}


def oracle_sample(wl, budget_s=12.0, max_steps=30):
    """Oracle throughput and final velocity on a bounded sample of the workload."""
    import oracle as O
    nx = wl.get("nx") or wl["n"]
    p = O.Params(wl["n"], wl["L"], wl["nu"], wl["eta"], O.MEAN_FIXED, nx=nx, Lx=wl["L"] * nx / wl["n"])
    ins = O.Insect.from_dict(wl["insect"]) if wl["insect"] else None
    ctl = O.StepControl(dt_fixed=wl["dt_fixed"], cfl=wl["cfl"] or 0.1, eta_cap=0.5)
    st = O.init_state(p, wl["u0"])
    st, _ = O.step(p, st, ctl, ins)  # first step (also warms scipy's plan cache)
    t0 = time.perf_counter()
    k = 0
    while k < max_steps and (time.perf_counter() - t0) < budget_s:
        st, _ = O.step(p, st, ctl, ins)
        k += 1
    dt = time.perf_counter() - t0
    return dict(steps=k + 1, timed_steps=k, seconds=dt, cores=O.flusi_oracle._WORKERS,
                u=O.velocity(p, st))


def error_vs_oracle(F, torch, wl, cs):
    """Relative L2 error of both precisions against the oracle's velocity after
    the oracle sample's step count (whole field and fluctuation about the mean)."""
    errs = {}
    for dtype in ("f32", "f64"):
        P = F.Plan(wl["n"], wl["L"], wl["nu"], wl["eta"], dtype, nx=wl.get("nx"))
        st = P.new_state(torch.from_numpy(wl["u0"]))
        P.step(st, cs["steps"], wl["insect"], dt_fixed=wl["dt_fixed"], cfl=wl["cfl"], eta_cap=0.5)
        u = P.velocity(st).double().cpu().numpy()
        ou = cs["u"]
        errs[dtype] = float(np.linalg.norm(u - ou) / np.linalg.norm(ou))
        fl = u - u.mean(axis=(1, 2, 3), keepdims=True)
        ofl = ou - ou.mean(axis=(1, 2, 3), keepdims=True)
        errs[dtype + "_fluct"] = float(np.linalg.norm(fl - ofl) / np.linalg.norm(ofl))
    return {"steps": cs["steps"], "rel_l2_f32": errs["f32"], "rel_l2_f64": errs["f64"],
            "rel_l2_fluct_f32": errs["f32_fluct"], "rel_l2_fluct_f64": errs["f64_fluct"]}


def measure(F, torch, name, wl, steps, warmup, tune):
    """FP32 and FP64 runs of one workload: FP32 throughput (`value`), the FP64
    figure, the dominant kernel's roofline (live per-pass HIP events on the
    launch stream, algorithmic bytes of the pruned model) and the step's."""
    n = wl["n"]
    nx = wl.get("nx") or n
    pts = float(nx) * n * n
    res = {}
    for dtype in ("f32", "f64"):
        res[dtype] = gpu_run(F, torch, wl, dtype, steps, warmup, tune=tune)
        note(f"{name} {dtype}: {res[dtype]['ev_ms'] / steps:.4f} ms/step")

    def mps(r):
        return pts * steps / (r["ev_ms"] / 1e3) / 1e6

    v32, v64 = mps(res["f32"]), mps(res["f64"])
    # dominant kernel of the FP32 run
    r = res["f32"]
    names = list(F.PASS_NAMES)
    split = r["pass_cnt"][names.index("z_inverse")] > 1
    pb = pass_bytes(n, 8, split, r["schedule"]["x_pass"], nx=nx)
    passes = {}
    for i, nm in enumerate(names):
        if r["pass_cnt"][i]:
            avg = r["pass_ms"][i] / r["pass_cnt"][i]
            passes[nm] = dict(avg_us=round(avg * 1e3, 3), launches=int(r["pass_cnt"][i]),
                              bytes=int(pb.get(nm, 0)), gbs=round(pb.get(nm, 0) / (avg * 1e-3) / 1e9, 1))
    step_names = ["y_inverse", "x_pass", "y_forward", "z_pass"] + (["z_inverse"] if split else [])
    ins = wl["insect"]
    nc = 0 if ins is None else (3 if ins.get("wings") else 1)
    dom = max(step_names, key=lambda k: r["pass_ms"][names.index(k)])
    d_avg_s = r["pass_ms"][names.index(dom)] / r["pass_cnt"][names.index(dom)] / 1e3
    achieved = pb[dom] / d_avg_s / 1e9
    sb = step_bytes(n, 8, nx=nx)
    return {
        "value": round(v32, 2),
        "ms_per_step": round(res["f32"]["ev_ms"] / steps, 5),
        "fp64": {"value": round(v64, 2), "unit": "Mpoint-steps/s",
                 "ms_per_step": round(res["f64"]["ev_ms"] / steps, 5),
                 "fp32_over_fp64": round(v32 / v64, 3)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic(name, kernel_of_pass(dom, n, "float", r["schedule"], nc,
                                                                     dyn=moving_body(ins), nx=nx)),
                     "algorithmic_bytes": int(pb[dom])},
        "step_roofline": {"bytes_per_step": sb, "bytes_per_point_step": round(sb / pts, 2),
                          "achieved_gbs": round(sb / (res["f32"]["ev_ms"] / steps / 1e3) / 1e9, 1),
                          "frac": round(sb / (res["f32"]["ev_ms"] / steps / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "passes_f32": passes,
        "schedule": {"f32": res["f32"]["schedule"], "f64": res["f64"]["schedule"],
                     "chosen_by": "autotune" if tune else "default"},
        "wall_s": {k: round(v["wall_s"], 4) for k, v in res.items()},
        "last_diag_f32": {"t": res["f32"]["diag"][0], "dt": res["f32"]["diag"][1],
                          "umax": res["f32"]["diag"][2], "drag": res["f32"]["diag"][4]},
    }


# ---------------------------------------------------------------------------
# Profile summaries: rocprofv3 output of one workload -> profiles/<workload>.md
# ---------------------------------------------------------------------------
PROFILE_STEPS = {"box1152": (10, 4), "ensemble48": (100, 20)}  # (trace steps, counter steps); default (100, 20)
SQ_SETS = ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_LDS_BANK_CONFLICT "
           "SQ_ACTIVE_INST_VALU",
           "SQ_WAVES SQ_ACTIVE_INST_LDS SQ_WAIT_INST_LDS SQ_ACTIVE_INST_ANY SQ_WAIT_INST_ANY SQ_INSTS_VMEM_RD "
           "SQ_INSTS_VMEM_WR SQ_INSTS_VALU")


def profile_commands(w: str, d: str = "gpurun_out/prof") -> list:
    """rocprofv3 command lines behind a workload's summary (run from the
    repository root, in this order: the trace run writes the schedule file
    that the counter runs reuse)."""
    s1, s2 = PROFILE_STEPS.get(w, (100, 20))
    skip = "--no-cpu --no-sphere --no-ensemble --no-serve --no-sponge --no-freeflight --no-rk4 --no-box"
    a = {"ensemble48": "--workload ensemble48", "box1152": f"--workload box1152 --warmup 2 {skip}"}.get(
        w, f"--workload {w} --warmup 5 {skip}")
    sf = f"--schedule-file {d}/sched_{w}.json"
    cmds = [f"rocprofv3 --kernel-trace --stats --output-format csv -d {d}/trace_{w} -o run -- "
            f"python3 bench.py {a} --steps {s1} {sf}"]
    for tag, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        cmds.append(f"rocprofv3 --pmc {ctr} --output-format csv -d {d}/{tag}_{w} -o run -- "
                    f"python3 bench.py {a} --steps {s2} {sf}")
    if w in ("insect256", "sphere128"):
        for i, ctr in enumerate(SQ_SETS):
            cmds.append(f"rocprofv3 --pmc {ctr} --output-format csv -d {d}/sq{i + 1}_{w} -o run -- "
                        f"python3 bench.py {a} --steps {s2} {sf}")
    for tag, ctr in (("copy_fetch", "FETCH_SIZE"), ("copy_write", "WRITE_SIZE")):
        cmds.append(f"rocprofv3 --pmc {ctr} --output-format csv -d {d}/{tag} -o run -- "
                    f"python3 bench.py --copy-calibration")
    cmds.append(f"python3 bench.py --summarize {d} --workload {w} > profiles/{w}.md")
    return cmds


def short_kernel(name: str) -> str:
    """Kernel name without return type, namespace and parameter list."""
    import re
    name = re.sub(r"^void ", "", name.strip()).replace("flusi::", "")
    depth = 0
    for i, ch in enumerate(name):
        depth += ch == "<"
        depth -= ch == ">"
        if ch == "(" and depth == 0:
            return name[:i]
    return name


def alg_bytes(kernel: str):
    """Algorithmic HBM bytes per member of a launch of a stepping kernel (the
    model of pass_bytes), or None for kernels outside the step."""
    import re
    m = re.match(r"(k_xpass|k_ypass|k_zpass)<(float|double), (\d+), (\d+), (-?\d+), (-?\d+), (\w+)>", kernel)
    if not m:
        return None
    fam, real, nx, n, a, b, c = m.groups()
    nx, n, a, b = int(nx), int(n), int(a), int(b)
    cb = 8 if real == "float" else 16
    if fam == "k_xpass":
        return None if c == "true" else pass_bytes(n, cb, False, x_variant=b, nx=nx)["x_pass"]
    if fam == "k_ypass":
        return pass_bytes(n, cb, False, nx=nx)["y_inverse" if a == 1 else "y_forward"]
    if a in (1, 2):
        return pass_bytes(n, cb, split_z=(a == 2), nx=nx)["z_pass"]
    if a == 3:
        return pass_bytes(n, cb, False, nx=nx)["z_inverse"]
    return None


def _rows(path: str):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def summarize(d: str, w: str) -> str:
    """Markdown summary of the rocprofv3 runs of workload w under directory d."""
    from collections import defaultdict

    def wg(r, g="Grid_Size", b="Workgroup_Size"):
        gs = int(r.get(g) or r.get(g + "_X"))
        return gs // max(1, int(r.get(b) or r.get(b + "_X")))

    def calib(tag, ctr):
        v = [float(r["Counter_Value"]) for r in _rows(f"{d}/{tag}/run_counter_collection.csv")
             if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer") and r["Counter_Name"] == ctr
             and float(r["Counter_Value"]) > 1e5]
        return sum(v) / len(v), (1 << 30) / 1024 / (sum(v) / len(v))

    cf, sf = calib("copy_fetch", "FETCH_SIZE")
    cw, sw = calib("copy_write", "WRITE_SIZE")
    trace = defaultdict(list)
    for r in _rows(f"{d}/trace_{w}/run_kernel_trace.csv"):
        trace[(short_kernel(r["Kernel_Name"]), wg(r))].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    ctr = defaultdict(lambda: defaultdict(list))
    for tag in ("fetch", "write", "sq1", "sq2"):
        p = f"{d}/{tag}_{w}/run_counter_collection.csv"
        if os.path.exists(p):
            for r in _rows(p):
                ctr[(short_kernel(r["Kernel_Name"]), wg(r))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    mean = lambda v: sum(v) / len(v) if v else None
    total = sum(sum(v) for v in trace.values())
    # one-member grid of each kernel: every launch of a solo workload; in the
    # ensemble run, the smallest grid of a kernel also launched one by one
    # (kernels seen at one grid only there, e.g. autotune variants: unknown)
    per_member, grids = {}, defaultdict(set)
    for (k, g) in trace:
        per_member[k] = min(per_member.get(k, g), g)
        grids[k].add(g)
    if w == "ensemble48":
        per_member = {k: g for k, g in per_member.items() if len(grids[k]) > 1}
    with open(f"{d}/trace_{w}.json") as f:
        line = json.loads(f.read())
    desc = line.get("config", {}).get("description", "")
    out = [f"# rocprofv3 summary: {w} ({desc})", "", f"csrc_sha256: {source_hash()}", "",
           "Commands (repository root, MI355X; the first writes the schedule file the others reuse):", ""]
    out += [f"    {c}" for c in profile_commands(w)]
    out += ["", f"Copy calibration (1 GiB device copy, `__amd_rocclr_copyBuffer`): FETCH_SIZE reads {cf:.0f} KiB "
            f"(scale x{sf:.3f}), WRITE_SIZE reads {cw:.0f} KiB (scale x{sw:.3f}).", "",
            "Rows are split by launch grid (workgroups); members = grid / the kernel's smallest grid in the run "
            "(one member).  alg = the algorithmic bytes of the pass model (bench.py pass_bytes) times members; "
            "HBM = FETCH_SIZE and WRITE_SIZE scaled by the copy calibration; GB/s and frac use alg bytes and "
            "the average duration against 8 TB/s."
            + ("  The size groups run concurrently on their own streams, so a grouped launch's duration "
               "includes sharing the GPU with the other groups' launches (the durations add up to more than "
               "the wall time); the one-member rows come from the one-by-one comparison leg."
               if w == "ensemble48" else ""), "",
            "| kernel | grid | members | calls | avg us | % time | alg MB | HBM read MB | HBM write MB | HBM/alg | alg GB/s | frac |",
            "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    traffic = []
    for (k, g), ts in sorted(trace.items(), key=lambda kv: -sum(kv[1])):
        pct = 100.0 * sum(ts) / total
        avg = sum(ts) / len(ts)
        mem = g // per_member[k] if (k in per_member and g % per_member[k] == 0) else None
        ab = alg_bytes(k)
        ab = ab * mem if (ab is not None and mem) else None
        c = ctr.get((k, g), {})
        fb = mean(c.get("FETCH_SIZE", [])) * 1024 * sf if c.get("FETCH_SIZE") else None
        wb = mean(c.get("WRITE_SIZE", [])) * 1024 * sw if c.get("WRITE_SIZE") else None
        if (pct < 0.05 and ab is None) or (pct < 0.3 and fb is None):
            continue  # autotune trials and one-off set-up launches
        fmt = lambda x, p=2: "-" if x is None else f"{x:.{p}f}"
        ratio = (fb + wb) / ab if (ab and fb is not None and wb is not None) else None
        gbs = ab / (avg * 1e-6) / 1e9 if ab else None
        out.append(f"| `{k}` | {g} | {mem or '-'} | {len(ts)} | {avg:.2f} | {pct:.2f} | {fmt(ab and ab / 1e6)} | "
                   f"{fmt(fb and fb / 1e6)} | {fmt(wb and wb / 1e6)} | {fmt(ratio, 3)} | {fmt(gbs, 1)} | "
                   f"{fmt(gbs and gbs / HBM_PEAK_GBS, 3)} |")
        if mem == 1 and fb is not None and wb is not None:
            traffic.append(f"traffic {k} {int(fb)} {int(wb)}")
    sq = [(k, c) for k, c in ctr.items() if "SQ_WAVES" in c and alg_bytes(k[0]) is not None]
    if sq:
        out += ["", "## SQ counters (per launch averages; ratios per wave or per wave-cycle)", "",
                "Instruction counts are per wave; the active and wait columns divide SQ_ACTIVE_INST_* and "
                "SQ_WAIT_INST_* by SQ_WAVE_CYCLES (the same quad-cycle units), i.e. the fraction of a wave's "
                "lifetime spent issuing or waiting; LDS conflict = SQ_LDS_BANK_CONFLICT cycles per LDS "
                "instruction.", "",
                "| kernel | grid | waves | VALU/wave | SALU/wave | LDS/wave | LDS conflict cyc/LDS inst | "
                "VALU active/wave-cyc | LDS active/wave-cyc | LDS wait/wave-cyc | any wait/wave-cyc | "
                "VMEM rd/wave | VMEM wr/wave |", "|---|---:|" + "---:|" * 11]
        for (k, g), c in sorted(sq, key=lambda kc: -sum(trace.get(kc[0], [0]))):
            m = {n: mean(v) for n, v in c.items()}
            wv = m.get("SQ_WAVES") or 1
            cyc = m.get("SQ_WAVE_CYCLES")
            r = lambda n, dnm: "-" if m.get(n) is None or not dnm else f"{m[n] / dnm:.3g}"
            out.append(f"| `{k}` | {g} | {wv:.0f} | {r('SQ_INSTS_VALU', wv)} | {r('SQ_INSTS_SALU', wv)} | "
                       f"{r('SQ_INSTS_LDS', wv)} | {r('SQ_LDS_BANK_CONFLICT', m.get('SQ_INSTS_LDS'))} | "
                       f"{r('SQ_ACTIVE_INST_VALU', cyc)} | {r('SQ_ACTIVE_INST_LDS', cyc)} | "
                       f"{r('SQ_WAIT_INST_LDS', cyc)} | {r('SQ_WAIT_INST_ANY', cyc)} | "
                       f"{r('SQ_INSTS_VMEM_RD', wv)} | {r('SQ_INSTS_VMEM_WR', wv)} |")
    rf = line.get("roofline")
    if rf:
        sch = line["schedule"]["f32"]
        ins_nc = {"insect256": 3, "box1152": 3}.get(w, 1)
        n = line["config"].get("grid")
        k = kernel_of_pass(rf["kernel"], n, "float", sch, ins_nc, dyn=w in ("insect256", "box1152", "freefall128"),
                           nx=line["config"].get("nx"))
        dyn = w in ("insect256", "box1152", "freefall128")
        ts = trace.get((k, per_member.get(k, -1)), [])
        if ts:
            out += ["", f"Dominant kernel of the bench line ({rf['kernel']}, `{k}`): HIP events "
                    f"{line['passes_f32'][rf['kernel']]['avg_us']:.2f} us per launch, rocprofv3 "
                    f"{sum(ts) / len(ts):.2f} us ({len(ts)} launches)."]
        # one FP32 step of the timed schedule: its pass kernels against the bench's step time
        names = ["y_inverse", "x_pass", "y_forward", "z_pass"] + (["z_inverse"] if sch["split_z"] else [])
        ks = [kernel_of_pass(p_, n, "float", sch, ins_nc, dyn=dyn, nx=line["config"].get("nx")) for p_ in names]
        avgs = [trace.get((k_, per_member.get(k_, -1)), []) for k_ in ks]
        if all(avgs):
            tot_us = sum(sum(a_) / len(a_) for a_ in avgs)
            sb = step_bytes(n, 8, nx=line["config"].get("nx"))
            out += [f"FP32 step of the timed schedule: its pass kernels average {tot_us:.1f} us together "
                    f"(rocprofv3), the bench line {line['ms_per_step'] * 1e3:.1f} us per step; {sb / 1e6:.1f} MB "
                    f"algorithmic per step = {sb / (tot_us * 1e-6) / 1e9:.0f} GB/s over the kernel time "
                    f"({sb / (tot_us * 1e-6) / 1e9 / HBM_PEAK_GBS:.3f} of peak)."]
    out += ["", "## bench.py line of the trace run", "", "```json", json.dumps(line), "```", "",
            "## Traffic per launch used by bench.py (scaled counters, bytes; one-member launches)", "", "```"]
    out += sorted(traffic) + ["```", ""]
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="insect256",
                    choices=["sphere128", "freefall128", "insect256", "box192", "box1152", "tg32", "ensemble48",
                             "serve"])
    ap.add_argument("--no-sphere", action="store_true", help="skip the 128^3 sphere figure")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-stream figure")
    ap.add_argument("--no-sponge", action="store_true", help="skip the vorticity-sponge figure")
    ap.add_argument("--no-freeflight", action="store_true", help="skip the free-flight figure")
    ap.add_argument("--no-rk4", action="store_true", help="skip the RK4 figure")
    ap.add_argument("--no-box", action="store_true", help="skip the non-cubic box figure")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble figure")
    ap.add_argument("--no-autotune", action="store_true", help="time the default schedules")
    ap.add_argument("--summarize", default=None, metavar="DIR",
                    help="print the profiles/ summary of --workload from the rocprofv3 runs under DIR")
    ap.add_argument("--schedule-file", default=None,
                    help="JSON file of schedules: reused when present, else written from this run's choices")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 1 GiB (3 launches) to scale HBM counters")
    a = ap.parse_args()
    if a.summarize:
        print(summarize(a.summarize, a.workload))
        return
    if a.schedule_file:
        SCHED_PIN["path"] = a.schedule_file
        if os.path.exists(a.schedule_file):
            with open(a.schedule_file) as f:
                SCHED_PIN["data"] = json.load(f)
    if a.copy_calibration:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4, "launches": 3}))
        return
    if a.gpus != 1:
        print(f"bench.py: the solver runs on one GPU (asked for {a.gpus}); its fields are not "
              "decomposed over several GPUs", file=sys.stderr)
        raise SystemExit(2)

    import torch
    import paper_1506_06513_amd as F

    if a.workload == "ensemble48":
        e = ensemble_run(F, torch, steps=a.steps or 200, tune=not a.no_autotune)
        print(json.dumps({"metric": METRIC, "value": e["value"], "unit": e["unit"], "n_gpus": 1,
                          "steps": e["steps"], "warmup": e["graph_chunk"], "ms_per_step": round(e["ms"] / e["steps"], 5),
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                          "data": "synthetic", "config": {"workload": "ensemble48", "description": e["description"]},
                          "ensemble": e}), flush=True)
        return

    if a.workload == "serve":
        sv = serve_run(F, torch)
        sv["saturated"] = serve_run(F, torch, saturate=True)
        print(json.dumps({"metric": METRIC, "value": sv["value"], "unit": sv["unit"], "n_gpus": 1,
                          "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": "serve", "description": sv["description"]},
                          "p50_ms": sv["p50_ms"], "p99_ms": sv["p99_ms"], "serving": sv}), flush=True)
        return

    wl = build_workload(a.workload)
    steps = a.steps or wl["default_steps"]
    n = wl["n"]
    nx = wl.get("nx") or n
    pts = float(nx) * n * n
    out = {
        "metric": METRIC,
        "value": None,
        "unit": "Mpoint-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": a.workload, "description": wl["desc"], "grid": n, **({"nx": nx} if nx != n else {})},
    }
    m = measure(F, torch, a.workload, wl, steps, a.warmup, not a.no_autotune)
    out["value"] = m.pop("value")
    out["ms_per_step"] = m.pop("ms_per_step")
    out.update(m)
    extras = a.workload == "insect256"
    swl = build_workload("sphere128") if extras else wl
    s_steps = swl["default_steps"] if extras else steps
    if extras and not a.no_sphere:
        ms = measure(F, torch, "sphere128", swl, s_steps, a.warmup, not a.no_autotune)
        out["sphere128"] = dict(ms, steps=s_steps, description=swl["desc"])
        if not a.no_cpu:
            out["sphere128"]["err_vs_oracle"] = error_vs_oracle(F, torch, swl, oracle_sample(swl, budget_s=5.0))
        note("sphere128 done")
    spts = float(swl["n"]) ** 3
    if not a.no_ensemble and extras:
        out["ensemble48"] = ensemble_run(F, torch, tune=not a.no_autotune)
        note("ensemble48 done")
    if not a.no_serve and extras:
        out["serving"] = serve_run(F, torch)
        note("serving done")
        out["serving"]["saturated"] = serve_run(F, torch, saturate=True)
        note("saturated serving done")
    if not a.no_sponge and extras:
        # the same workload with a vorticity sponge layer 3.5 <= x < 4 (C_sp = 0.1)
        sp = {}
        for dtype in ("f32", "f64"):
            r = gpu_run(F, torch, swl, dtype, s_steps, a.warmup, tune=not a.no_autotune,
                        sponge=(0.1, (0.5, 0.0, 0.0)))
            sp[dtype] = round(spts * s_steps / (r["ev_ms"] / 1e3) / 1e6, 2)
        note("sponge done")
        out["sponge"] = {"value": sp["f32"], "fp64": sp["f64"], "unit": "Mpoint-steps/s",
                         "description": "sphere128 with the vorticity sponge on 3.5 <= x < 4, C_sp = 0.1 "
                                        "(3 more forward fields per step)"}
    if not a.no_freeflight and extras:
        # the same workload with the sphere in free flight
        import workloads as W
        ff_body = W.free_sphere(swl["insect"])
        ff = {}
        for dtype in ("f32", "f64"):
            r = gpu_run(F, torch, dict(swl, insect=ff_body), dtype, s_steps, a.warmup, tune=not a.no_autotune)
            ff[dtype] = (round(spts * s_steps / (r["ev_ms"] / 1e3) / 1e6, 2), r["diag"])
        d = ff["f32"][1]
        note("free flight done")
        out["freeflight"] = {"value": ff["f32"][0], "fp64": ff["f64"][0], "unit": "Mpoint-steps/s",
                             "description": "sphere128 with the sphere in free flight (density 2, g = 1 along -z, "
                                            "6 DoF): 13-value body state advanced each step",
                             "body_at_last_step_f32": {"t": d[0], "x_cntr": list(d[22:25]), "u_cntr": list(d[25:28]),
                                                       "omega_b": list(d[32:35])}}
    if not a.no_rk4 and extras:
        # the same workload with the RK4 integrator (explicit diffusion, 4 stages per step)
        rk = {}
        for dtype in ("f32", "f64"):
            r = gpu_run(F, torch, swl, dtype, max(10, s_steps // 4), a.warmup, tune=not a.no_autotune,
                        integrator="rk4")
            rk[dtype] = round(spts * max(10, s_steps // 4) / (r["ev_ms"] / 1e3) / 1e6, 2)
        note("rk4 done")
        out["rk4"] = {"value": rk["f32"], "fp64": rk["f64"], "unit": "Mpoint-steps/s",
                      "description": "sphere128 stepped with classical RK4 and explicit diffusion "
                                     "(four pipeline passes per step)"}
    if not a.no_box and extras:
        # the paper's own box at its own resolution: FP32 and FP64, few steps
        bw = build_workload("box1152")
        bpts = 1152.0 * 768 * 768
        bv = {}
        for dtype in ("f32", "f64"):
            r = gpu_run(F, torch, bw, dtype, bw["default_steps"], 2, tune=not a.no_autotune)
            bv[dtype] = round(bpts * bw["default_steps"] / (r["ev_ms"] / 1e3) / 1e6, 2)
            torch.cuda.empty_cache()
        note("box1152 done")
        out["box1152"] = {"value": bv["f32"], "fp64": bv["f64"], "unit": "Mpoint-steps/s",
                          "steps": bw["default_steps"], "description": bw["desc"]}
        # the sphere workload in the 6x4x4 box shape of the paper at 192x128x128 points
        bx = build_workload("box192")
        bpts = 192.0 * 128 * 128
        bv = {}
        for dtype in ("f32", "f64"):
            r = gpu_run(F, torch, bx, dtype, s_steps, a.warmup, tune=not a.no_autotune)
            bv[dtype] = round(bpts * s_steps / (r["ev_ms"] / 1e3) / 1e6, 2)
        note("box done")
        out["box192"] = {"value": bv["f32"], "fp64": bv["f64"], "unit": "Mpoint-steps/s",
                         "description": "192x128x128 box 6x4x4 (one spacing 1/32), sphere R=0.5 at (2.4, 2, 2), "
                                        "inflow (1,0,0) + noise rms 1e-3 (seed 0), nu=0.01, C_eta=1e-3, CFL 0.1"}
    if not a.no_cpu:
        note("cpu baseline (oracle) running")
        cs = oracle_sample(wl)
        cpu_v = pts * cs["timed_steps"] / cs["seconds"] / 1e6
        out["cpu_baseline"] = {"value": round(cpu_v, 3), "unit": "Mpoint-steps/s", "cores": cs["cores"],
                               "kind": "oracle",
                               "sample": f"{cs['timed_steps']} steps of the same workload after 1 untimed step "
                                         f"({cs['seconds']:.1f} s, NumPy/SciPy FP64)"}
        out["err_vs_oracle"] = error_vs_oracle(F, torch, wl, cs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

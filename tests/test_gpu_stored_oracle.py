"""Full-size workloads against stored oracle results (needs an MI355X).

At these sizes the oracle takes minutes to an hour, so its results come from
files under tests/golden/, each written by the script beside it, which calls
only the oracle and the seeded input generators.  A file holds the time, step
size and max |u| of each step, each part's force and torque at each step
(body, left wing, right wing), and the velocity at 2048 seeded grid points,
half of them around the insect.  The GPU runs the same steps from the same
seeded input and is compared with them element by element, within the bars of
the 100-step parity tests (FP64 and FP32):

- insect512_turbulent.txt (make_insect512.py): the large request of the
  serving stream, the 512^3 model insect (nu = 1/136, C_eta = 2.5e-4) in
  k^(-5/3) turbulent inflow (intensity 0.1, 1 <= |k| <= 32, mean (1, 0, 0),
  seed 2), two steps at CFL 0.1 with dt <= C_eta/2;
- insect256_100.txt (make_insect256.py): the headline workload, the flapping
  model insect in the 256^3 box from rest, 100 steps with the same controls;
- box192_100.txt, freefall128_100.txt, sponge128_100.txt and rk4_128_100.txt
  (make_sphere_workloads.py): the benchmark's sphere in inflow with noise in
  the 192x128x128 box, and at 128^3 in free flight (the body state is compared
  too), with the vorticity sponge, and stepped with RK4; 100 steps each."""
import os
import sys

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


def _golden(golden_dir, name, with_solid=False):
    rows = [l.split() for l in open(os.path.join(golden_dir, name)) if not l.startswith("#")]
    steps = np.array([[float(v) for v in r[1:4]] for r in rows if r[0] == "step"])
    forces = np.array([[float(v) for v in r[2:8]] for r in rows if r[0] == "force"])
    forces = forces.reshape(len(steps), len(forces) // len(steps), 6)
    pts = np.array([[int(v) for v in r[1:4]] for r in rows if r[0] == "u"])
    vel = np.array([[float(v) for v in r[4:7]] for r in rows if r[0] == "u"])
    if with_solid:
        solid = np.array([[float(v) for v in r[1:]] for r in rows if r[0] == "solid"])
        return steps, forces, pts, vel, (solid[0] if len(solid) else None)
    return steps, forces, pts, vel


def _run(n, L, u0, dtype, nsteps, pts, body=None, nu=1.0 / 136.0, eta=2.5e-4, nx=None, sponge=None,
         integrator="ab2"):
    """GPU steps (CFL 0.1, dt <= C_eta/2) of the body (default: the model
    insect, nu = 1/136, C_eta = 2.5e-4) from u0; the step history, the velocity
    at the grid points pts (i, j, k) and the body state."""
    P = F.Plan(n, L, nu, eta, dtype, nx=nx) if nx else F.Plan(n, L, nu, eta, dtype)
    if sponge is not None:
        P.set_sponge(*sponge)
    P.set_integrator(integrator)
    st = P.new_state(u0)
    body = W.model_insect(n, L) if body is None else body
    h = P.step(st, nsteps, body, history=True, cfl=0.1, eta_cap=0.5).detach().cpu().numpy()
    assert P.forces(st)[0] == 0
    solid = np.asarray(P.solid(st)) if body.get("free_flight") else None
    u = P.velocity(st)
    i, j, k = (torch.from_numpy(pts[:, a]).to(u.device) for a in range(3))
    gvel = u[:, k, j, i].T.double().cpu().numpy()
    del u, P, st
    torch.cuda.empty_cache()
    return h, gvel, solid


def _check_history(h, steps, forces, tol_dt, tol_umax, tol_f, first):
    assert np.allclose(h[:, 0], steps[:, 0], rtol=tol_dt, atol=0)
    assert np.allclose(h[:, 1], steps[:, 1], rtol=tol_dt, atol=0)
    assert np.allclose(h[:, 2], steps[:, 2], rtol=tol_umax, atol=0)
    # per-part force and torque (body, left wing, right wing) from step `first`
    for c in range(forces.shape[1]):
        gF, gM = h[first:, 4 + 6 * c:7 + 6 * c], h[first:, 7 + 6 * c:10 + 6 * c]
        oF, oM = forces[first:, c, :3], forces[first:, c, 3:]
        assert np.max(np.abs(gF - oF)) <= tol_f * np.max(np.abs(oF)), c
        assert np.max(np.abs(gM - oM)) <= tol_f * np.max(np.abs(oM)), c


# max point error / max |u|; relative bars of dt, max |u| and the forces
TOL512 = {"f64": (1e-11, 1e-12, 1e-12, 1e-9), "f32": (2e-5, 1e-6, 2e-5, 1e-3)}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_insect512_turbulent_inflow_two_steps_match_the_oracle(golden_dir, dtype):
    tol_u, tol_dt, tol_umax, tol_f = TOL512[dtype]
    steps, forces, pts, ovel = _golden(golden_dir, "insect512_turbulent.txt")
    n, L = 512, 4.0
    u0 = torch.from_numpy(W.turbulent_inflow(n, L, seed=2, intensity=0.1, kmin=1.0, kmax=32.0))
    h, gvel, _ = _run(n, L, u0, dtype, len(steps), pts)
    err = np.max(np.abs(gvel - ovel)) / np.max(np.abs(ovel))
    print(f"insect512 turbulent {dtype}, 2 steps: max point error / max |u| = {err:.3e}")
    assert err <= tol_u
    _check_history(h, steps, forces, tol_dt, tol_umax, tol_f, 0)


# relative L2 over the sampled points; relative bars of dt, max |u| and the forces
TOL256 = {"f64": (1e-11, 1e-12, 1e-11, 1e-9), "f32": (2e-5, 1e-6, 2e-5, 1e-3)}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_insect256_hundred_steps_match_the_oracle(golden_dir, dtype):
    tol_u, tol_dt, tol_umax, tol_f = TOL256[dtype]
    steps, forces, pts, ovel = _golden(golden_dir, "insect256_100.txt")
    n, L = 256, 4.0
    u0 = torch.zeros((3, n, n, n), dtype=torch.float64)
    h, gvel, _ = _run(n, L, u0, dtype, len(steps), pts)
    err = float(np.linalg.norm(gvel - ovel) / np.linalg.norm(ovel))
    print(f"insect256 {dtype}, 100 steps: relative L2 over the sampled points = {err:.3e}")
    assert err <= tol_u
    # the first step starts from a fluid at rest: its forces have no
    # unsteady term and are compared from the second step on, as at 128^3
    _check_history(h, steps, forces, tol_dt, tol_umax, tol_f, 1)


# the benchmark's sphere workloads (make_sphere_workloads.py): relative L2 over
# the sampled points; relative bars of dt, max |u|, the force and the body state
TOLSPH = {"f64": (1e-11, 1e-12, 1e-11, 1e-9, 1e-11), "f32": (2e-5, 1e-6, 2e-5, 1e-3, 2e-5)}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", ["box192_100", "freefall128_100", "sponge128_100", "rk4_128_100"])
def test_sphere_workloads_hundred_steps_match_the_oracle(golden_dir, name, dtype):
    sys.path.insert(0, golden_dir)
    import make_sphere_workloads as M
    tol_u, tol_dt, tol_umax, tol_f, tol_s = TOLSPH[dtype]
    steps, forces, pts, ovel, osolid = _golden(golden_dir, f"{name}.txt", with_solid=True)
    nx, n, _, free = M.CASES[name]
    u0 = torch.from_numpy(M.case_input(name))
    h, gvel, solid = _run(n, M.L, u0, dtype, len(steps), pts, body=M.case_body(name), nu=M.NU, eta=M.ETA,
                          nx=nx if nx != n else None, sponge=M.case_sponge(name),
                          integrator=M.case_integrator(name))
    err = float(np.linalg.norm(gvel - ovel) / np.linalg.norm(ovel))
    print(f"{name} {dtype}, {len(steps)} steps: relative L2 over the sampled points = {err:.3e}")
    assert err <= tol_u
    _check_history(h, steps, forces, tol_dt, tol_umax, tol_f, 0)
    if free:
        assert np.max(np.abs(solid - osolid)) <= tol_s * max(1.0, np.max(np.abs(osolid)))

"""Writes the oracle's results for the benchmark's sphere workloads after 100
steps (CFL 0.1, dt <= C_eta / 2; nu = 0.01, C_eta = 1e-3; inflow (1, 0, 0) plus
solenoidal noise of rms 1e-3 on |k| <= 8, seed 0; a sphere of radius 0.5):

- box192_100.txt: the 192x128x128 box (6 x 4 x 4), the sphere at (2.4, 2, 2);
- freefall128_100.txt: the 128^3 box, the sphere at the centre in free flight
  (density 2, gravity 1 along -z, six degrees of freedom);
- sponge128_100.txt: the 128^3 box with the vorticity sponge on 3.5 <= x < 4
  (C_sp = 0.1, Sec. 2.3);
- rk4_128_100.txt: the 128^3 box stepped with RK4 (Sec. 2.4) instead of AB2.

Each file holds the time, step size and max |u| of every step, the body's
force and torque at every step, and the velocity at 2048 seeded grid points
(half of them drawn from the box around the sphere); the free-flight file also
holds the 13-value body state after the steps.  The script calls only the oracle
and the seeded input generators; about an hour on 8 host cores for all cases
(names as arguments select some):

    python tests/golden/make_sphere_workloads.py [name ...]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

L, NU, ETA, STEPS, NPTS = 4.0, 0.01, 1e-3, 100, 2048

CASES = {
    # name: (nx, n, body centre, free flight)
    "box192_100": (192, 128, (2.4, 2.0, 2.0), False),
    "freefall128_100": (128, 128, (2.0, 2.0, 2.0), True),
    "sponge128_100": (128, 128, (2.0, 2.0, 2.0), False),
    "rk4_128_100": (128, 128, (2.0, 2.0, 2.0), False),
}
# the vorticity sponge of the sponge case: C_sp and the layer thickness per axis
SPONGE = (0.1, (0.5, 0.0, 0.0))


def case_integrator(name: str) -> str:
    return "rk4" if name.startswith("rk4") else "ab2"


def case_sponge(name: str):
    return SPONGE if name.startswith("sponge") else None


def case_body(name: str) -> dict:
    nx, n, xc, free = CASES[name]
    body = dict(W.sphere_body(L), x_cntr=xc)
    return W.free_sphere(body) if free else body


def case_input(name: str) -> np.ndarray:
    nx, n, xc, free = CASES[name]
    return W.inflow_noise(n, L, seed=0, rms=1e-3, kmax=8.0, nx=nx if nx != n else None)


def sample_points(nx: int, n: int, xc) -> np.ndarray:
    """(NPTS, 3) grid indices (i, j, k) = (x, y, z): half anywhere, half in the
    cube of side 2 about the sphere's starting centre."""
    rng = np.random.default_rng(nx * 1000 + n)
    dx = L / n
    anywhere = np.stack([rng.integers(0, nx, NPTS // 2), rng.integers(0, n, NPTS // 2),
                         rng.integers(0, n, NPTS // 2)], axis=1)
    m = NPTS - NPTS // 2
    near = np.stack([rng.integers(int((c - 1.0) / dx), int((c + 1.0) / dx), m) for c in xc], axis=1)
    return np.concatenate([anywhere, near])


def main():
    for name, (nx, n, xc, free) in CASES.items():
        if len(sys.argv) > 1 and name not in sys.argv[1:]:
            continue
        kw = dict(nx=nx, Lx=L * nx / n) if nx != n else {}
        kw["integrator"] = case_integrator(name)
        if case_sponge(name):
            kw.update(c_sp=case_sponge(name)[0], sponge=tuple(case_sponge(name)[1]))
        p = O.Params(n, L, NU, ETA, O.MEAN_FIXED, **kw)
        ins = O.Insect.from_dict(case_body(name))
        st, hist = O.run(p, case_input(name), STEPS, O.StepControl(cfl=0.1, eta_cap=0.5), ins)
        u = O.velocity(p, st)
        pts = sample_points(nx, n, xc)
        out = os.path.join(HERE, f"{name}.txt")
        with open(out, "w") as f:
            f.write(f"# oracle (tests/golden/make_sphere_workloads.py): {name}, {STEPS} steps, CFL 0.1,\n")
            f.write("# dt <= C_eta/2; rows: 'step t dt umax', 'force 0 Fx Fy Fz Mx My Mz' (the sphere),\n")
            f.write("# 'solid' and the 13-value body state after the steps (free flight only), then\n")
            f.write("# 'u i j k ux uy uz' at grid points x = i dx, y = j dx, z = k dx after the steps\n")
            for d in hist:
                f.write(f"step {d['t']!r} {d['dt']!r} {d['umax']!r}\n")
                vals = list(d["F"][0]) + list(d["M"][0])
                f.write("force 0 " + " ".join(repr(float(v)) for v in vals) + "\n")
            if free:
                f.write("solid " + " ".join(repr(float(v)) for v in st.solid) + "\n")
            for i, j, k in pts:
                vals = u[:, k, j, i]
                f.write(f"u {i} {j} {k} " + " ".join(repr(float(v)) for v in vals) + "\n")
        print("wrote", out, flush=True)


if __name__ == "__main__":
    main()

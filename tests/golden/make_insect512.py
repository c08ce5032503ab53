"""Writes insect512_turbulent.txt: the oracle's result for the large request of
the serving stream, the 512^3 model insect (nu = 1/136, C_eta = 2.5e-4) in
k^(-5/3) turbulent inflow (intensity 0.1, 1 <= |k| <= 32, mean (1, 0, 0),
seed 2), after two steps of Algorithm 1 (CFL 0.1, dt <= C_eta / 2): the time,
step size and max |u| of each step, each part's force and torque, and the
velocity at 2048 seeded grid points (half of them drawn from the box around the
insect).  It calls only the oracle and the seeded input generators; it needs
about 50 GB of memory and a few minutes:

    python tests/golden/make_insect512.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

N, L, NU, ETA, SEED, STEPS = 512, 4.0, 1.0 / 136.0, 2.5e-4, 2, 2
NPTS = 2048


def sample_points(n: int, L: float) -> np.ndarray:
    """(NPTS, 3) grid indices (i, j, k) = (x, y, z): half anywhere, half in the
    cube of side 2.4 about the box centre, where the insect is."""
    rng = np.random.default_rng(512)
    anywhere = rng.integers(0, n, size=(NPTS // 2, 3))
    dx = L / n
    lo, hi = int((L / 2 - 1.2) / dx), int((L / 2 + 1.2) / dx)
    near = rng.integers(lo, hi, size=(NPTS - NPTS // 2, 3))
    return np.concatenate([anywhere, near])


def main():
    u0 = W.turbulent_inflow(N, L, seed=SEED, intensity=0.1, kmin=1.0, kmax=32.0)
    p = O.Params(N, L, NU, ETA, O.MEAN_FIXED)
    ins = O.Insect.from_dict(W.model_insect(N, L))
    st, hist = O.run(p, u0, STEPS, O.StepControl(cfl=0.1, eta_cap=0.5), ins)
    del u0
    u = O.velocity(p, st)
    pts = sample_points(N, L)
    out = os.path.join(HERE, "insect512_turbulent.txt")
    with open(out, "w") as f:
        f.write("# oracle (tests/golden/make_insect512.py): 512^3 model insect in turbulent inflow,\n")
        f.write("# two steps, CFL 0.1, dt <= C_eta/2; rows: 'step t dt umax', 'force c Fx Fy Fz Mx My Mz'\n")
        f.write("# (c = body, left wing, right wing; moments about each part's reference point),\n")
        f.write("# then 'u i j k ux uy uz' at grid points x = i dx, y = j dx, z = k dx after the steps\n")
        for s, d in enumerate(hist):
            f.write(f"step {d['t']!r} {d['dt']!r} {d['umax']!r}\n")
            for c in range(3):
                vals = list(d["F"][c]) + list(d["M"][c])
                f.write("force " + str(c) + " " + " ".join(repr(float(v)) for v in vals) + "\n")
        for i, j, k in pts:
            vals = u[:, k, j, i]
            f.write(f"u {i} {j} {k} " + " ".join(repr(float(v)) for v in vals) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()

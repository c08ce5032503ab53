"""Writes insect256_100.txt: the oracle's result for the headline workload, the
flapping model insect in the 256^3 box (L = 4, nu = 1/136, C_eta = 2.5e-4,
fluid at rest), after 100 steps of Algorithm 1 (CFL 0.1, dt <= C_eta / 2): the
time, step size and max |u| of every step, each part's force and torque at
every step, and the velocity at 2048 seeded grid points (half of them drawn
from the box around the insect).  It calls only the oracle and the seeded input
generators; it needs about 6 GB of memory and half an hour:

    python tests/golden/make_insect256.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

N, L, NU, ETA, STEPS = 256, 4.0, 1.0 / 136.0, 2.5e-4, 100
NPTS = 2048


def sample_points(n: int, L: float) -> np.ndarray:
    """(NPTS, 3) grid indices (i, j, k) = (x, y, z): half anywhere, half in the
    cube of side 2.4 about the box centre, where the insect is."""
    rng = np.random.default_rng(256)
    anywhere = rng.integers(0, n, size=(NPTS // 2, 3))
    dx = L / n
    lo, hi = int((L / 2 - 1.2) / dx), int((L / 2 + 1.2) / dx)
    near = rng.integers(lo, hi, size=(NPTS - NPTS // 2, 3))
    return np.concatenate([anywhere, near])


def main():
    u0 = np.zeros((3, N, N, N))
    p = O.Params(N, L, NU, ETA, O.MEAN_FIXED)
    ins = O.Insect.from_dict(W.model_insect(N, L))
    st, hist = O.run(p, u0, STEPS, O.StepControl(cfl=0.1, eta_cap=0.5), ins)
    u = O.velocity(p, st)
    pts = sample_points(N, L)
    out = os.path.join(HERE, "insect256_100.txt")
    with open(out, "w") as f:
        f.write("# oracle (tests/golden/make_insect256.py): 256^3 flapping model insect, fluid at rest,\n")
        f.write("# 100 steps, CFL 0.1, dt <= C_eta/2; rows: 'step t dt umax', 'force c Fx Fy Fz Mx My Mz'\n")
        f.write("# (c = body, left wing, right wing; moments about each part's reference point),\n")
        f.write("# then 'u i j k ux uy uz' at grid points x = i dx, y = j dx, z = k dx after the steps\n")
        for d in hist:
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

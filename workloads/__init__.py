"""Seeded synthetic inputs and workload definitions.

Shared by the tests and the benchmark for both the HIP library and the oracle.
It holds none of the solver's arithmetic: it only samples initial velocity
fields and lists the parameters of each workload as plain numbers.

Workloads (shapes follow the paper's dimensionless scales: K = sqrt(nu C_eta)/dx
near 0.1, stroke amplitude 140 deg, Re 100-500, C_eta 1e-4..1e-3):

  tg32       32^3, L = 2 pi, 2D Taylor-Green vortex embedded in 3D, no mask,
             nu = 0.01, fixed dt = 1e-3, 100 steps (closed-form decay).
  sphere128  128^3, L = 4, fixed sphere of radius 0.5 at the box centre with a
             tanh mask of width 2 dx, mean inflow (1,0,0), nu = 0.01,
             C_eta = 1e-3, solenoidal noise of rms 1e-3 in |k| <= 8,
             adaptive dt at CFL 0.1, 500 steps.
  insect256  256^3, L = 4, ellipsoid body (0.5, 0.1, 0.1) and two flat
             elliptic wings (span 1, chord 0.35, thickness 4 dx), stroke
             +-70 deg, feathering +-45 deg shifted by pi/2, frequency 1,
             nu = 1/136, C_eta = 2.5e-4, CFL 0.1, fluid at rest.
  ensemble   insect simulations on {64,96,128,192}^3 with seeded Re, C_eta
             and stroke amplitude.
  serve      Poisson-arrival request stream (mean 4 per s): one 512^3 insect
             in isotropic k^(-5/3) turbulent inflow (intensity 0.1,
             1 <= |k| <= 32, 2000 steps) arriving second, and ensemble-like
             insect requests (200 steps, fluid at rest).
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft

DEG = math.pi / 180.0


def grid_axis(n: int, L: float) -> np.ndarray:
    return np.arange(n, dtype=np.float64) * (L / n)


def taylor_green(n: int, L: float = 2.0 * math.pi) -> np.ndarray:
    """u = (sin x cos y, -cos x sin y, 0) sampled on the grid, [3][z][y][x]."""
    a = grid_axis(n, L)
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    u = np.zeros((3, n, n, n))
    u[0] = np.sin(x) * np.cos(y)
    u[1] = -np.cos(x) * np.sin(y)
    return u


def _random_solenoidal(n: int, seed: int, kmin: float, kmax: float, slope: float | None, nx: int | None = None):
    """Random-phase band-limited divergence-free field (unit-free amplitude) on
    an nx x n x n grid with one spacing (nx = n: cubic).

    Each Fourier mode with kmin <= |j| <= kmax gets a random vector made
    perpendicular to j (cross product with j) and a random phase; with `slope`
    set, mode amplitudes follow an energy spectrum E(k) ~ k^slope.  On a
    longer x axis j_x is counted in units of the y and z axes' base
    wavenumber (j_x n / nx)."""
    nx = n if nx is None else nx
    rng = np.random.default_rng(seed)
    jx = np.arange(nx // 2 + 1)[None, None, :]
    js = np.arange(n)
    js = np.where(js < n // 2, js, js - n)
    jy = js[None, :, None]
    jz = js[:, None, None]
    shape = (n, n, nx // 2 + 1)
    jxf = np.broadcast_to(jx, shape).astype(np.float64) * (n / nx)
    jyf = np.broadcast_to(jy, shape).astype(np.float64)
    jzf = np.broadcast_to(jz, shape).astype(np.float64)
    kmag = np.sqrt(jxf ** 2 + jyf ** 2 + jzf ** 2)
    shell = (kmag >= kmin) & (kmag <= kmax)
    r = rng.standard_normal((3,) + shape)
    a = np.stack([r[1] * jzf - r[2] * jyf, r[2] * jxf - r[0] * jzf, r[0] * jyf - r[1] * jxf])
    norm = np.sqrt(np.sum(a * a, axis=0))
    norm = np.where(norm > 0, norm, 1.0)
    amp = np.ones(shape)
    if slope is not None:
        kk = np.where(kmag > 0, kmag, 1.0)
        # |a|^2 per mode ~ E(k) / (shell area ~ k^2)
        amp = np.sqrt(kk ** slope / kk ** 2)
    phase = np.exp(2j * math.pi * rng.random(shape))
    coef = a / norm * amp * phase * shell
    return scipy.fft.irfftn(coef, s=(n, n, nx), axes=(1, 2, 3), workers=os.cpu_count())


def inflow_noise(n: int, L: float, seed: int, rms: float = 1e-3, kmax: float = 8.0,
                 mean=(1.0, 0.0, 0.0), nx: int | None = None) -> np.ndarray:
    """Mean inflow plus random-phase solenoidal noise in 1 <= |k| <= kmax, scaled
    so that the rms of |u'| equals `rms`; [3][n][n][nx] with nx = n by default."""
    del L
    up = _random_solenoidal(n, seed, 1.0, kmax, None, nx)
    s = math.sqrt(float(np.mean(np.sum(up * up, axis=0))))
    up *= rms / s
    up[0] += mean[0]
    up[1] += mean[1]
    up[2] += mean[2]
    return up


def turbulent_inflow(n: int, L: float, seed: int, intensity: float = 0.1, kmin: float = 1.0,
                     kmax: float = 32.0, mean=(1.0, 0.0, 0.0)) -> np.ndarray:
    """Mean inflow plus random-phase isotropic turbulence with E(k) ~ k^(-5/3)
    on kmin <= |k| <= kmax; per-component rms = intensity * |mean|."""
    del L
    up = _random_solenoidal(n, seed, kmin, kmax, -5.0 / 3.0)
    s = math.sqrt(float(np.mean(np.sum(up * up, axis=0))) / 3.0)
    umag = math.sqrt(sum(m * m for m in mean))
    up *= intensity * umag / s
    for c in range(3):
        up[c] += mean[c]
    return up


def random_bandlimited(n: int, seed: int, kmax: float, solenoidal: bool = True) -> np.ndarray:
    """Random physical field with modes |k| <= kmax (test input)."""
    if solenoidal:
        return _random_solenoidal(n, seed, 1.0, kmax, None) * n ** 1.5
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3, n, n, n))


# --------------------------------------------------------------------------
# Workload parameter sets (plain numbers)
# --------------------------------------------------------------------------

def sphere_body(L: float = 4.0, radius: float = 0.5) -> dict:
    return dict(body="sphere", x_cntr=(L / 2, L / 2, L / 2), radius=radius,
                smooth="tanh", c_smth=1.0)


def free_sphere(body: dict) -> dict:
    """The sphere of a workload in free flight: density 2 (twice the fluid's),
    gravity 1 along -z, all six degrees of freedom, J = (2/5) M R^2."""
    r = body.get("radius", 0.5)
    mass = 2.0 * 4.0 / 3.0 * math.pi * r ** 3
    return dict(body, free_flight=True, mass=mass, inertia=(0.4 * mass * r * r,) * 3, gravity=1.0,
                dof=(1, 1, 1, 1, 1, 1))


def model_insect(n: int, L: float = 4.0, phi_m: float = 70.0 * DEG,
                 alpha_m: float = 45.0 * DEG) -> dict:
    """Tethered model insect at the box centre: horizontal stroke plane
    (pitch -45 deg, stroke-plane angle -45 deg), pivots 0.15 from the axis."""
    return dict(body="ellipsoid", x_cntr=(L / 2, L / 2, L / 2),
                psi=0.0, beta=-45.0 * DEG, gamma=0.0,
                a=0.5, b=0.1, smooth="cos", c_smth=1.0,
                wings=True, eta_stroke=-45.0 * DEG,
                pivot_l=(0.0, 0.15, 0.0), pivot_r=(0.0, -0.15, 0.0),
                wing_A=0.175, wing_B=0.5, wing_t=4.0 * L / n,
                freq=1.0, phi=(0.0, phi_m, 0.0), alpha=(0.0, alpha_m, -math.pi / 2),
                theta=(0.0, 0.0, 0.0))


WORKLOADS = {
    "tg32": dict(n=32, L=2.0 * math.pi, nu=0.01, eta=1.0, mean_mode=1,
                 steps=100, dt_fixed=1e-3, cfl=0.0, insect=None),
    "sphere128": dict(n=128, L=4.0, nu=0.01, eta=1e-3, mean_mode=0,
                      steps=500, dt_fixed=0.0, cfl=0.1, insect="sphere", seed=0),
    "insect256": dict(n=256, L=4.0, nu=1.0 / 136.0, eta=2.5e-4, mean_mode=0,
                      steps=None, t_end=1.0, dt_fixed=0.0, cfl=0.1, insect="insect"),
}


def ensemble_members(count: int = 48, seed: int = 1, grids=(64, 96, 128, 192), L: float = 4.0):
    """Seeded insect ensemble: grid, Re in [50,500], C_eta in [1e-4,1e-3],
    stroke amplitude in [50,80] deg, feathering 45 deg."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(grids[int(rng.integers(0, len(grids)))])
        re = float(rng.uniform(50.0, 500.0))
        eta = float(rng.uniform(1e-4, 1e-3))
        phim = float(rng.uniform(50.0, 80.0)) * DEG
        out.append(dict(id=i, n=n, L=L, nu=1.0 / re, eta=eta, phi_m=phim,
                        insect=model_insect(n, L, phi_m=phim)))
    return out


def serve_stream(count: int = 120, seed: int = 2, rate: float = 4.0, big_n: int = 512, big_steps: int = 2000,
                 small_steps: int = 200, L: float = 4.0):
    """Request list of the serving workload with arrival times in seconds.

    Arrivals: Poisson process of the given mean rate (first arrival at 0).
    Request 1 is the large insect in turbulent inflow (its initial field is
    `turbulent_inflow(big_n, L, seed)`, built by the caller); the others are
    drawn like the ensemble members and start from rest."""
    rng = np.random.default_rng(seed + 1000)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.concatenate([[0.0], np.cumsum(gaps[1:])])
    small = ensemble_members(count - 1, seed=seed, L=L)
    out = []
    for i in range(count):
        if i == 1:
            out.append(dict(id=i, arrival=float(arrivals[i]), n=big_n, L=L, nu=1.0 / 136.0, eta=2.5e-4,
                            steps=big_steps, insect=model_insect(big_n, L), turbulent=True, seed=seed))
        else:
            m = small[i if i == 0 else i - 1]
            out.append(dict(id=i, arrival=float(arrivals[i]), n=m["n"], L=L, nu=m["nu"], eta=m["eta"],
                            steps=small_steps, insect=m["insect"], turbulent=False))
    return out

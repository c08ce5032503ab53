"""Pins of the oracle's non-cubic boxes (Sec. 4 and 6: a 6x4x4 box at
1152x768x768 points, one spacing on every axis): the per-axis wavenumber scale
(a Laplacian eigenmode decays at its own rate), the 2/3 rule per axis, and
periodic images (a cubic run tiled along x equals the run in the longer box,
with energy and forces doubled)."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def test_box_geometry_and_two_thirds_rule_per_axis():
    g = O.Grid(32, 4.0, 48, 6.0)
    assert g.shape == (32, 32, 48) and g.dx == 0.125 and g.dV == 0.125 ** 3
    x, y, z = g.coords()
    assert x.shape == (32, 32, 48) and x.max() == 6.0 - 0.125 and y.max() == 4.0 - 0.125
    keep = g.dealias()
    # kept: |jx| <= 15 (3*15 < 48 <= 3*16), |jy|, |jz| <= 10 (3*10 < 32 <= 3*11)
    assert keep.shape == (32, 32, 25) and int(keep.sum()) == 16 * 21 * 21
    jx, jy, jz = g.wavenumbers()
    assert np.all(keep == ((jx <= 15) & (np.abs(jy) <= 10) & (np.abs(jz) <= 10)))
    kx, ky, kz = g.k_vectors(derivative=False)
    assert kx[0, 0, 1] == 2 * math.pi / 6.0 and ky[0, 1, 0] == 2 * math.pi / 4.0
    with pytest.raises(ValueError):
        O.Grid(32, 4.0, 48, 5.0)  # unequal spacing


def _cell(g, a_j, b_j):
    """u = (sin(ax) cos(by), -(a/b) cos(ax) sin(by), 0): a Laplacian
    eigenfunction's velocity, so u x w is a gradient and the field decays at
    exp(-nu (a^2 + b^2) t)."""
    x, y, _ = g.coords()
    a, b = 2 * math.pi / g.Lx * a_j, 2 * math.pi / g.L * b_j
    u = np.zeros((3,) + g.shape)
    u[0] = np.sin(a * x) * np.cos(b * y)
    u[1] = -(a / b) * np.cos(a * x) * np.sin(b * y)
    return u, a * a + b * b


def test_eigenmode_decays_at_its_own_rate_in_a_long_box():
    n, L, nx, Lx, nu, dt, steps = 16, 4.0, 24, 6.0, 0.05, 0.02, 25
    p = O.Params(n, L, nu, 1.0, O.MEAN_FREE, nx=nx, Lx=Lx)
    u0, k2 = _cell(O.grid_of(p), 2, 1)
    st, hist = O.run(p, u0, steps, O.StepControl(dt_fixed=dt))
    assert np.max(np.abs(O.velocity(p, st) - math.exp(-nu * k2 * dt * steps) * u0)) < 1e-13
    g = O.grid_of(p)
    assert abs(hist[0]["E"] - 0.5 * float(np.sum(u0 * u0)) * g.dV) < 1e-13
    # a wrong x scale (2 pi / L instead of 2 pi / Lx) would give this rate instead
    wrong = (2 * math.pi / L * 2) ** 2 + (2 * math.pi / L) ** 2
    assert abs(math.exp(-nu * wrong * dt * steps) - math.exp(-nu * k2 * dt * steps)) > 1e-2


def test_tiled_run_equals_cubic_run_with_a_body():
    """The cubic n^3 run with a sphere, tiled twice along x, equals the run in
    the 2n x n x n box with the two-sphere mask (the doubled box keeps exactly
    the even-jx modes' 2/3 rule); energy and forces double."""
    n, L, nu, eta, steps = 16, 4.0, 0.02, 1e-2, 6
    u0 = W.inflow_noise(n, L, seed=5, rms=0.05, kmax=4.0)
    p1 = O.Params(n, L, nu, eta, O.MEAN_FIXED)
    g1 = O.grid_of(p1)
    ins = O.Insect.from_dict(W.sphere_body(L, radius=0.8))
    chi, us, col = O.insect_mask(g1, ins, 0.0)
    xref = O.reference_points(ins, 0.0)
    st1, h1 = O.run(p1, u0, steps, O.StepControl(cfl=0.2), fixed_mask=(chi, us, col, xref))
    p2 = O.Params(n, L, nu, eta, O.MEAN_FIXED, nx=2 * n, Lx=2 * L)
    tile = lambda f: np.concatenate([f, f], axis=-1)
    st2, h2 = O.run(p2, tile(u0), steps, O.StepControl(cfl=0.2),
                    fixed_mask=(tile(chi), tile(us), tile(col), xref))
    assert np.max(np.abs(O.velocity(p2, st2) - tile(O.velocity(p1, st1)))) < 1e-13
    for a, b in zip(h1, h2):
        assert a["dt"] == b["dt"]
        assert abs(b["E"] - 2 * a["E"]) < 1e-12 * a["E"]
        assert np.max(np.abs(b["F"] - 2 * a["F"])) < 1e-11 * np.max(np.abs(a["F"]))


def test_layers_follow_the_axis_lengths():
    g = O.Grid(16, 4.0, 24, 6.0)
    chi = O.sponge_mask(g, (0.5, 0.0, 0.5))
    x, y, z = g.coords()
    assert np.array_equal(chi > 0, (x >= 5.5) | (z >= 3.5))

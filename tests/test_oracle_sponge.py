"""Pins of the oracle's vorticity sponge (Sec. 2.3, eq. PNST_org_momentum).

The sponge term -(1/C_sp) curl(chi_sp w)/Laplacian is read as the Biot-Savart
damping of the vorticity: with chi_sp = 1 everywhere it must equal -u/C_sp for
a divergence-free field (damping at rate 1/C_sp), it must be divergence-free
for any layer, and it must leave the mean flow (k = 0) alone."""
import math

import numpy as np

import oracle as O
import workloads as W


def _grid(n=24, L=2 * math.pi):
    return O.Grid(n, L)


def test_layer_placement():
    g = _grid(16, 4.0)
    chi = O.sponge_mask(g, (0.5, 0.0, 1.0))
    x, y, z = g.coords()
    want = ((x >= 3.5) | (z >= 3.0)).astype(float)
    assert np.array_equal(chi, want)
    assert np.array_equal(O.sponge_mask(g, (0.0, 0.0, 0.0)), np.zeros_like(x))


def test_full_sponge_damps_at_rate_one_over_csp():
    g = _grid()
    u = W.random_bandlimited(g.n, 3, kmax=5.0)
    uh = O.import_field(g, u)
    w = O.c2r(O.curl_hat(g, uh), g.n)
    c_sp = 0.1
    s = O.sponge_hat(g, w, np.ones_like(w[0]), c_sp)
    ref = -uh / c_sp
    ref[:, 0, 0, 0] = 0.0
    assert np.max(np.abs(s - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_sponge_term_is_divergence_free_and_leaves_the_mean():
    g = _grid(32, 4.0)
    rng = np.random.default_rng(4)
    w = rng.standard_normal((3, g.n, g.n, g.n))
    s = O.sponge_hat(g, w, O.sponge_mask(g, (1.0, 0.5, 0.0)), 0.2)
    div = O.divergence_hat(g, s)
    kx, ky, kz = g.k_vectors(derivative=True)
    kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
    assert np.max(np.abs(div)) <= 1e-14 * np.max(kmag * np.abs(s).max(axis=0))
    assert np.all(s[:, 0, 0, 0] == 0.0)


def test_taylor_green_with_full_sponge_follows_the_ifab2_recurrence():
    # u x w is a gradient for the Taylor-Green field, so the right-hand side is
    # the sponge alone: N_hat = -u_hat/C_sp on its |k|^2 = 2 modes.  The run
    # must follow the scalar IF-AB2 recurrence with lambda = -1/C_sp.
    n, L, nu, c_sp = 24, 2 * math.pi, 0.02, 0.05
    g = O.Grid(n, L)
    p = O.Params(n, L, nu, 1.0, O.MEAN_FREE, c_sp=c_sp, sponge=(L, 0.0, 0.0))
    u0 = W.taylor_green(n)
    dts = [2e-3, 3e-3, 1.5e-3, 2.5e-3]
    st = O.init_state(p, u0)
    for dt in dts:
        st, _ = O.step(p, st, O.StepControl(dt_fixed=dt), None)
    lam, k2 = -1.0 / c_sp, 2.0
    a, a_prev, n_prev, dt_prev = 1.0, None, None, None
    for i, dt in enumerate(dts):
        nn = lam * a
        if i == 0:
            a_new = math.exp(-nu * k2 * dt) * (a + dt * nn)
        else:
            r = dt / dt_prev
            a_new = math.exp(-nu * k2 * dt) * (a + dt * ((1 + r / 2) * nn - (r / 2) * math.exp(-nu * k2 * dt_prev) * n_prev))
        n_prev, dt_prev, a = nn, dt, a_new
    u = O.velocity(p, st)
    assert np.max(np.abs(u - a * u0)) <= 1e-13 * np.max(np.abs(u0))


def test_no_sponge_when_switched_off():
    g = _grid(16, 4.0)
    uh = O.import_field(g, W.random_bandlimited(16, 2, kmax=4.0))
    p0 = O.Params(16, 4.0, 0.01, 1.0, O.MEAN_FREE)
    p1 = O.Params(16, 4.0, 0.01, 1.0, O.MEAN_FREE, c_sp=0.1, sponge=(0.0, 0.0, 0.0))
    a, _ = O.rhs_hat(p0, g, uh, None, None)
    b, _ = O.rhs_hat(p1, g, uh, None, None)
    assert np.array_equal(a, b)

"""Pins of the oracle's right-hand side and AB2-IF time stepping (CPU only).

P5 Taylor-Green closed form, P6 energy invariant of the rotational form,
P7 exact AB2-IF recurrence against its characteristic roots, P8 second
order with variable steps, dt rule checks."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def test_taylor_green_closed_form_decay():
    # u x w = -grad(sin^2 x sin^2 y) is a resolved gradient, so the projected
    # right-hand side vanishes and every mode decays as exp(-2 nu t).
    p = O.Params(32, 2 * math.pi, 0.01, 1.0, O.MEAN_FREE)
    u0 = W.taylor_green(32)
    st, hist = O.run(p, u0, 100, O.StepControl(dt_fixed=1e-3))
    assert st.t == pytest.approx(0.1, abs=1e-15)
    u = O.velocity(p, st)
    ex = u0 * math.exp(-2 * 0.01 * st.t)
    assert np.linalg.norm(u - ex) / np.linalg.norm(ex) < 1e-13
    assert math.exp(-0.002) == pytest.approx(0.998002, abs=1e-6)
    # <|u|^2> = <sin^2 x cos^2 y + cos^2 x sin^2 y> = 1/2, so E(0) = (1/2)(1/2)(2 pi)^3,
    # and the energy history follows exp(-4 nu t)
    e0 = hist[0]["E"]
    assert e0 == pytest.approx(0.5 * 0.5 * (2 * math.pi) ** 3, rel=1e-13)
    for h in hist[::10]:
        assert h["E"] == pytest.approx(e0 * math.exp(-4 * 0.01 * h["t"]), rel=1e-12)


def test_rotational_form_conserves_energy():
    # For nu = 0 and chi = 0, sum_k w Re(u_hat^* . N_hat) = 0: u.(u x w) = 0
    # pointwise, Parseval, and the projection is self-adjoint and fixes u_hat.
    n = 24
    p = O.Params(n, 2 * math.pi, 0.0, 1.0, O.MEAN_FREE)
    g = O.Grid(n, p.L)
    u0 = W.random_bandlimited(n, 3, kmax=7.0)
    uh = O.import_field(g, u0)
    nh, _ = O.rhs_hat(p, g, uh, None, None)
    w = np.full(uh.shape[-1], 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    dot = float(np.sum(w * np.real(np.conj(uh) * nh)))
    scale = float(np.sum(w * np.abs(uh) * np.abs(nh)))
    assert scale > 0
    assert abs(dot) <= 1e-13 * scale


def test_energy_drift_is_second_order():
    n = 16
    p = O.Params(n, 2 * math.pi, 0.0, 1.0, O.MEAN_FREE)
    u0 = W.random_bandlimited(n, 9, kmax=4.0)
    u0 *= 0.5 / np.sqrt(np.mean(np.sum(u0 * u0, axis=0)))
    drifts = []
    for dt in (0.02, 0.01, 0.005):
        steps = int(round(0.4 / dt))
        st, hist = O.run(p, u0, steps, O.StepControl(dt_fixed=dt))
        g = O.Grid(n, p.L)
        e1 = O.energy_spectral(g, st.uh)
        drifts.append(abs(e1 - hist[0]["E"]))
    r1, r2 = drifts[0] / drifts[1], drifts[1] / drifts[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5


def _relaxation_setup(n=16, eta=0.05, nu=0.1, amp=0.3):
    """chi = 1 everywhere, u_s = 0, single mode u = (0, A sin x, 0): the
    projected right-hand side is exactly -u_hat/C_eta."""
    L = 2 * math.pi
    p = O.Params(n, L, nu, eta, O.MEAN_FREE)
    a = W.grid_axis(n, L)
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    u0 = np.stack([0 * x, amp * np.sin(x), 0 * x])
    chi = np.ones((n, n, n))
    us = np.zeros((3, n, n, n))
    colour = np.ones((n, n, n), dtype=np.int16)
    xref = np.zeros((3, 3))
    return p, u0, (chi, us, colour, xref)


def test_ab2_if_matches_characteristic_roots():
    eta, nu, dt = 0.05, 0.1, 0.01
    p, u0, fm = _relaxation_setup(eta=eta, nu=nu)
    st, _ = O.run(p, u0, 40, O.StepControl(dt_fixed=dt), fixed_mask=fm)
    uy = O.velocity(p, st)[1]
    amp_num = uy[0, 0, 4] / math.sin(4 * 2 * math.pi / 16)
    # y_{n+1} = E[(1 + 3z/2) y_n - (z/2) E y_{n-1}],  y_1 = E(1 + z) y_0,
    # E = exp(-nu k^2 dt) with k = 1, z = -dt/C_eta: closed form from the roots
    E = math.exp(-nu * dt)
    zz = -dt / eta
    bq = E * (1 + 1.5 * zz)
    cq = 0.5 * zz * E * E
    disc = math.sqrt(bq * bq - 4 * cq)
    x1, x2 = (bq + disc) / 2, (bq - disc) / 2
    y0, y1 = 0.3, E * (1 + zz) * 0.3
    c2 = (y1 - x1 * y0) / (x2 - x1)
    c1 = y0 - c2
    exact = c1 * x1 ** 40 + c2 * x2 ** 40
    assert amp_num == pytest.approx(exact, rel=1e-12)


def _variable_dt_run(p, u0, fm, T, h):
    """Integrate with a non-uniform step pattern built from h (oracle pieces)."""
    g = O.Grid(p.n, p.L)
    chi, us, _, _ = fm
    uh = O.import_field(g, u0)
    t, n, nh_prev, dt_prev = 0.0, 0, None, None
    while t < T - 1e-14:
        dt = h * (1.0 + 0.4 * math.sin(1.7 * n))
        dt = min(dt, T - t)
        nh, _ = O.rhs_hat(p, g, uh, chi, us)
        uh = O.ab2_if(p, g, uh, nh, nh_prev, dt, dt_prev if nh_prev is not None else dt)
        nh_prev, dt_prev, t, n = nh, dt, t + dt, n + 1
    return O.c2r(uh, p.n)


def test_ab2_variable_step_is_second_order():
    eta, nu, amp = 0.5, 0.2, 0.3
    p, u0, fm = _relaxation_setup(eta=eta, nu=nu, amp=amp)
    T = 1.0
    exact = amp * math.exp(-(nu + 1.0 / eta) * T)
    errs = []
    for h in (0.04, 0.02, 0.01):
        uy = _variable_dt_run(p, u0, fm, T, h)[1]
        errs.append(abs(uy[0, 0, 4] / math.sin(4 * 2 * math.pi / 16) - exact))
    assert 3.2 < errs[0] / errs[1] < 5.0
    assert 3.2 < errs[1] / errs[2] < 5.0


def test_dt_rule():
    ctl = O.StepControl(cfl=0.1, eta_cap=0.5)
    assert O.choose_dt(ctl, 2.0, 0.05, 1e-3, False, 0.0) == pytest.approx(0.0025)
    assert O.choose_dt(ctl, 2.0, 0.05, 1e-3, True, 0.0) == pytest.approx(5e-4)
    assert O.choose_dt(O.StepControl(cfl=0.1, t_end=1.0), 1.0, 0.05, 1e-3, False, 0.999) == pytest.approx(0.001)
    assert O.choose_dt(O.StepControl(cfl=0.1, dt_max=1e-4), 1.0, 0.05, 1e-3, False, 0.0) == 1e-4
    assert O.choose_dt(O.StepControl(cfl=0.1), 0.0, 0.05, 1e-3, False, 0.0) == math.inf
    assert O.choose_dt(O.StepControl(dt_fixed=1e-3), 5.0, 0.05, 1e-3, True, 0.0) == 1e-3


def test_pure_relaxation_inside_solid_matches_exponential():
    # Sec. 2.1: with nonlinear, viscous and pressure terms set aside, du/dt = -u/C_eta
    # inside the solid.  The mean mode (k = 0) feels exactly that.
    n = 8
    eta = 0.1
    p = O.Params(n, 2 * math.pi, 0.3, eta, O.MEAN_FREE)
    u0 = np.zeros((3, n, n, n))
    u0[0] = 1.0
    fm = (np.ones((n, n, n)), np.zeros((3, n, n, n)), np.ones((n, n, n), np.int16), np.zeros((3, 3)))
    T = 0.5
    errs = []
    for dt in (0.01, 0.005):
        st, _ = O.run(p, u0, int(round(T / dt)), O.StepControl(dt_fixed=dt), fixed_mask=fm)
        errs.append(abs(O.velocity(p, st)[0].mean() - math.exp(-T / eta)))
    assert errs[1] < 1e-3 and 3.0 < errs[0] / errs[1] < 5.0

"""Pins of the oracle's RK4 integrator with explicit diffusion (Sec. 2.4): the
stability polynomial of the classical scheme on problems whose right-hand side
is exactly linear (Taylor-Green, relaxation inside a solid), fourth-order
convergence on a nonlinear field and with a time-dependent solid velocity
(stage times), and the explicit-diffusion step cap."""
import math

import numpy as np

import oracle as O
import workloads as W


def _r4(z):
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def test_taylor_green_follows_the_rk4_polynomial():
    """Taylor-Green: u x w is a gradient, so R = -nu|k|^2 u_hat with |k|^2 = 2
    and n steps multiply the field by R4(-2 nu dt)^n."""
    n, L, nu, dt, steps = 16, 2 * math.pi, 0.05, 0.05, 20
    p = O.Params(n, L, nu, 1.0, O.MEAN_FREE, integrator="rk4")
    u0 = W.taylor_green(n)
    st, hist = O.run(p, u0, steps, O.StepControl(dt_fixed=dt))
    u = O.velocity(p, st)
    assert np.max(np.abs(u - _r4(-2 * nu * dt) ** steps * u0)) < 1e-14
    # and the exact decay within the scheme's error
    assert np.max(np.abs(u - math.exp(-2 * nu * dt * steps) * u0)) < 1e-9
    assert hist[-1]["dt"] == dt


def test_relaxation_inside_solid_follows_the_rk4_polynomial():
    """chi = 1, u_s = 0, single shear mode: R = -(1/C_eta + nu) u_hat exactly."""
    from test_oracle_time import _relaxation_setup
    eta, nu, dt, steps = 0.05, 0.1, 0.01, 30
    p, u0, fm = _relaxation_setup(eta=eta, nu=nu)
    p.integrator = "rk4"
    st, _ = O.run(p, u0, steps, O.StepControl(dt_fixed=dt), fixed_mask=fm)
    lam = -(1.0 / eta + nu)
    assert np.max(np.abs(O.velocity(p, st) - _r4(lam * dt) ** steps * u0)) < 1e-14


def _order(p, u0, ins, T, dts):
    ref, _ = O.run(p, u0, int(round(T / (dts[-1] / 4))), O.StepControl(dt_fixed=dts[-1] / 4), ins)
    uref = O.velocity(p, ref)
    errs = []
    for dt in dts:
        st, _ = O.run(p, u0, int(round(T / dt)), O.StepControl(dt_fixed=dt), ins)
        errs.append(float(np.max(np.abs(O.velocity(p, st) - uref))))
    return errs


def test_fourth_order_on_a_nonlinear_field():
    n, L = 16, 2 * math.pi
    p = O.Params(n, L, 0.02, 1.0, O.MEAN_FREE, integrator="rk4")
    u0 = W.inflow_noise(n, L, seed=9, rms=0.5, kmax=4.0)
    e1, e2 = _order(p, u0, None, 0.4, [0.04, 0.02])
    assert e2 < 1e-6 and 13.0 < e1 / e2 < 19.0


def test_fourth_order_with_a_time_dependent_solid_velocity():
    """A sphere (smooth tanh layer) turning about two axes, so that
    u_s = Omega^(g)(t) x (x - x_c) changes smoothly in time, with a weak
    penalization (C_eta = 0.5): fourth order needs u_s of each stage's time (a
    solid velocity frozen at t^n would make the forcing first order).  Bodies
    with kinks in their signed distance (the ellipsoid's max, the cosine
    layer's C^1 ends) limit any scheme to about second order, so they are not
    used here."""
    n, L = 16, 4.0
    p = O.Params(n, L, 0.02, 0.5, O.MEAN_FIXED, integrator="rk4")
    ins = O.Insect(body="sphere", x_cntr=(2.0, 2.0, 2.0), radius=1.0, smooth="tanh", c_smth=2.0,
                   gamma_dot=2.0, psi_dot=3.0)
    u0 = W.inflow_noise(n, L, seed=10, rms=0.05, kmax=3.0)
    e1, e2 = _order(p, u0, ins, 0.2, [0.02, 0.01])
    assert e2 < 1e-8 and 13.0 < e1 / e2 < 19.0


def test_explicit_diffusion_caps_the_step():
    n, L, nu = 16, 2 * math.pi, 0.5
    p = O.Params(n, L, nu, 1.0, O.MEAN_FREE, integrator="rk4")
    g = O.Grid(n, L)
    K = (n - 1) // 3
    cap = O.RK4_VISC / (nu * 3 * K * K)
    assert abs(O.rk4_visc_cap(p, g) - cap) < 1e-15 * cap
    st, hist = O.run(p, W.taylor_green(n), 5, O.StepControl(cfl=10.0))
    assert all(abs(d["dt"] - cap) < 1e-15 for d in hist)
    p2 = O.Params(n, L, nu, 1.0, O.MEAN_FREE)
    _, h2 = O.run(p2, W.taylor_green(n), 1, O.StepControl(cfl=10.0))
    assert h2[0]["dt"] > cap  # AB2 with the integrating factor has no such cap

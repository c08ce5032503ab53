"""Pins of the oracle's Dirichlet wall layers (Sec. 2.3: the velocity imposed by
the volume penalization in layers at the domain borders): layer placement,
precedence over a body, exclusion from the body's force integrals, and the
relaxation to the imposed velocity at the rate 1/C_eta (second order in dt)."""
import math

import numpy as np

import oracle as O
import workloads as W


def test_layers_sit_at_the_top_end_of_the_axes_and_carry_colour_zero():
    n, L = 24, 4.0
    g = O.Grid(n, L)
    p = O.Params(n, L, 0.01, 1e-2, O.MEAN_FIXED, wall=(0.5, 0.0, 1.0), u_wall=(1.0, -0.5, 0.25))
    chi, us, col = O.apply_walls(p, g, None, None, None)
    x, y, z = g.coords()
    inside = (x >= L - 0.5) | (z >= L - 1.0)
    assert np.array_equal(chi > 0, inside) and np.all(chi[inside] == 1.0)
    assert np.all(us[0][inside] == 1.0) and np.all(us[1][inside] == -0.5) and np.all(us[2][inside] == 0.25)
    assert np.all(us[:, ~inside] == 0.0) and np.all(col == 0)
    # x index i is in the layer iff i*dx >= L - d: dx = 1/6, so i = 21, 22, 23
    assert int(inside[0, 0, :].sum()) == 3


def test_layers_take_precedence_over_a_body():
    n, L = 32, 4.0
    g = O.Grid(n, L)
    ins = O.Insect.from_dict(dict(W.sphere_body(L), x_cntr=(3.5, 2.0, 2.0), radius=0.6))
    chi, us, col = O.insect_mask(g, ins, 0.0)
    p = O.Params(n, L, 0.01, 1e-2, O.MEAN_FIXED, wall=(0.5, 0.0, 0.0), u_wall=(1.0, 0.0, 0.0))
    c2, u2, k2 = O.apply_walls(p, g, chi, us, col)
    x = g.coords()[0]
    lay = x >= L - 0.5
    assert np.all(c2[lay] == 1.0) and np.all(k2[lay] == 0) and np.all(u2[0][lay] == 1.0)
    assert np.array_equal(c2[~lay], chi[~lay]) and np.array_equal(k2[~lay], col[~lay])
    assert np.sum((col == 1) & lay) > 0  # the body did reach into the layer


def test_layers_do_not_enter_the_body_force():
    """First step (same velocity): a sphere's force with a layer away from it
    equals the force without the layer (cosine mask: chi is exactly 0 in the
    layer; a tanh tail would reach into it and be taken over by the layer)."""
    n, L = 24, 4.0
    u0 = W.inflow_noise(n, L, seed=3, rms=1e-2, kmax=4.0)
    ins = O.Insect.from_dict(dict(W.sphere_body(L), smooth="cos"))
    ctl = O.StepControl(cfl=0.1)
    p0 = O.Params(n, L, 0.01, 1e-2, O.MEAN_FIXED)
    p1 = O.Params(n, L, 0.01, 1e-2, O.MEAN_FIXED, wall=(0.5, 0.0, 0.0), u_wall=(1.0, 0.0, 0.0))
    _, d0 = O.step(p0, O.init_state(p0, u0), ctl, ins)
    _, d1 = O.step(p1, O.init_state(p1, u0), ctl, ins)
    assert np.array_equal(d0["F"], d1["F"]) and np.array_equal(d0["M"], d1["M"])


def test_full_layer_relaxes_to_the_wall_velocity():
    """A layer covering the box: a uniform field obeys du/dt = -(u - u_wall)/C_eta
    exactly (the mean mode, no nonlinear term), so it approaches
    u_wall + (u0 - u_wall) exp(-t/C_eta) at second order in dt (AB2)."""
    n, L, eta, T = 16, 2 * math.pi, 0.05, 0.2
    uw = np.array([1.0, -0.5, 0.25])
    u0 = np.zeros((3, n, n, n)) + np.array([0.2, 0.3, -0.1]).reshape(3, 1, 1, 1)
    errs = []
    for dt in (4e-3, 2e-3):
        p = O.Params(n, L, 0.01, eta, O.MEAN_FREE, wall=(L, 0.0, 0.0), u_wall=tuple(uw))
        st, _ = O.run(p, u0, int(round(T / dt)), O.StepControl(dt_fixed=dt))
        u = O.velocity(p, st)
        exact = uw + (np.array([0.2, 0.3, -0.1]) - uw) * math.exp(-T / eta)
        errs.append(float(np.max(np.abs(u - exact.reshape(3, 1, 1, 1)))))
    assert errs[1] < 2e-3 and 3.5 < errs[0] / errs[1] < 4.5


def test_layers_do_not_enter_the_free_body_torque():
    """A free-flying sphere (cosine mask) with a wall layer away from it: the
    total force and the torque about its centre that drive the body, and the
    body state after the first step, equal those without the layer."""
    n, L = 24, 4.0
    u0 = W.inflow_noise(n, L, seed=4, rms=1e-2, kmax=4.0)
    ins = O.Insect.from_dict(dict(W.sphere_body(L), smooth="cos", free_flight=True, mass=2.0,
                                  inertia=(0.1, 0.1, 0.1), gravity=1.0, psi_dot=0.0))
    ctl = O.StepControl(cfl=0.1)
    p0 = O.Params(n, L, 0.01, 1e-2, O.MEAN_FIXED)
    p1 = O.Params(n, L, 0.01, 1e-2, O.MEAN_FIXED, wall=(0.5, 0.0, 0.0), u_wall=(1.0, 0.0, 0.0))
    s0, d0 = O.step(p0, O.init_state(p0, u0), ctl, ins)
    s1, d1 = O.step(p1, O.init_state(p1, u0), ctl, ins)
    assert np.array_equal(d0["F_total"], d1["F_total"]) and np.array_equal(d0["m_cntr"], d1["m_cntr"])
    assert np.array_equal(s0.solid, s1.solid)
    assert np.max(np.abs(d0["m_cntr"])) > 0.0

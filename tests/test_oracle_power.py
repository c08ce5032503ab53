"""Pins of the oracle's inertial power of a wing (Sec. 3.5):
P_inert = W . (J W' + W x J W), W the wing's angular velocity in its own frame,
J its tensor of inertia there.  Checked against facts that do not come from the
oracle's formula: the closed form of a wing that only strokes about one axis,
the vanishing period mean of a periodic motion, the rate of change of the
wing's rotational kinetic energy 1/2 W . J W, and the norm of W, which no
change of frame alters."""
import math

import numpy as np

import oracle as O

J_GENERAL = (2.0e-3, 5.0e-4, 2.4e-3, 3.0e-4, -2.0e-4, 1.5e-4)  # Jxx, Jyy, Jzz, Jxy, Jxz, Jyz


def _insect(**kw):
    d = dict(wings=True, freq=1.3, eta_stroke=-0.6, wing_J=J_GENERAL,
             phi=(0.1, 1.2, 0.0), alpha=(0.05, 0.7, -1.2), theta=(0.0, 0.15, 0.4))
    d.update(kw)
    return O.Insect(**d)


def _fourier_insect():
    r = math.radians
    return _insect(kin="fourier", freq=0.9,
                   kin_phi=((0.0, r(70), r(4.0), 0.0), (0.0, 0.0, r(2.0), 0.0)),
                   kin_alpha=((0.0, 0.0, 0.0, r(3.0)), (0.0, r(45), 0.0, r(-2.0))),
                   kin_theta=((r(2.0), 0.0, r(3.0), 0.0), (0.0, r(1.0), 0.0, 0.0)))


def test_pure_stroke_about_one_axis_has_the_closed_form():
    """Only phi moves, phi = phi_m cos(w t): W = phi' e_x in the wing frame, so
    P_inert = J_xx phi' phi'' = J_xx phi_m^2 w^3 sin(w t) cos(w t) for any J
    (the off-diagonal entries and the gyroscopic term drop out); the mirrored
    right wing needs the same power."""
    pm, f = 1.1, 1.7
    w = 2 * math.pi * f
    ins = _insect(freq=f, phi=(0.0, pm, 0.0), alpha=(0.0, 0.0, 0.0), theta=(0.0, 0.0, 0.0))
    for t in np.linspace(0.0, 1.0 / f, 13):
        exact = J_GENERAL[0] * pm * pm * w ** 3 * math.sin(w * t) * math.cos(w * t)
        scale = J_GENERAL[0] * pm * pm * w ** 3
        for side in ("l", "r"):
            assert abs(O.inertial_power(ins, t, side) - exact) <= 1e-8 * scale, (t, side)


def test_feathering_and_deviation_alone_have_their_closed_forms():
    """Only alpha moves: W = alpha' e_y, P_inert = J_yy alpha' alpha''; only
    theta moves: W = -theta' e_z, P_inert = J_zz theta' theta''."""
    am, f = 0.8, 1.4
    w = 2 * math.pi * f
    still = (0.0, 0.0, 0.0)
    ins_a = _insect(freq=f, phi=still, alpha=(0.0, am, 0.3), theta=still)
    ins_t = _insect(freq=f, phi=still, alpha=still, theta=(0.0, am, 0.3))
    for t in np.linspace(0.0, 1.0 / f, 11):
        # a = am cos(w t + 0.3): a' a'' = am^2 w^3 sin cos
        sc = am * am * w ** 3 * math.sin(w * t + 0.3) * math.cos(w * t + 0.3)
        scale = am * am * w ** 3
        for side in ("l", "r"):
            assert abs(O.inertial_power(ins_a, t, side) - J_GENERAL[1] * sc) <= 1e-8 * J_GENERAL[1] * scale
            assert abs(O.inertial_power(ins_t, t, side) - J_GENERAL[2] * sc) <= 1e-8 * J_GENERAL[2] * scale


def test_period_mean_vanishes_for_periodic_motion():
    """A periodic motion returns the kinetic energy it took: the mean of
    P_inert over a period is zero (periodic trapezoid rule, spectrally
    accurate), while P_inert itself is not small."""
    for ins in (_insect(), _fourier_insect()):
        T = 1.0 / ins.freq
        ts = np.arange(256) * T / 256
        for side in ("l", "r"):
            p = np.array([O.inertial_power(ins, t, side) for t in ts])
            assert np.max(np.abs(p)) > 1e-3
            assert abs(p.mean()) <= 1e-9 * np.max(np.abs(p)), side


def test_inertial_power_is_the_rate_of_the_rotational_kinetic_energy():
    """W . (J W') = d/dt (1/2 W . J W) for a symmetric J, and W . (W x J W) = 0:
    P_inert equals the derivative of the kinetic energy, differentiated here
    by Richardson extrapolation of central differences of the energy."""
    for ins in (_insect(), _fourier_insect()):
        J = O.wing_inertia(ins)
        for side in ("l", "r"):
            def energy(t):
                W = O.omega_wing_w(ins, t, side)
                return 0.5 * float(W @ J @ W)
            for t in (0.07, 0.31, 0.52):
                h = 1e-3 / ins.freq
                d1 = (energy(t + h) - energy(t - h)) / (2 * h)
                d2 = (energy(t + h / 2) - energy(t - h / 2)) / h
                rate = (4 * d2 - d1) / 3
                p = O.inertial_power(ins, t, side)
                assert abs(p - rate) <= 1e-6 * max(abs(p), 1e-3), (side, t, p, rate)


def test_wing_frame_velocity_has_the_norm_of_the_body_frame_one():
    for ins in (_insect(), _fourier_insect()):
        for side in ("l", "r"):
            for t in (0.0, 0.2, 0.45):
                a = np.linalg.norm(O.omega_wing_w(ins, t, side))
                b = np.linalg.norm(O.omega_wing_b(ins, t, side))
                assert abs(a - b) <= 1e-14 * max(a, 1.0)


def test_no_inertia_means_no_inertial_power():
    ins = _insect(wing_J=(0.0,) * 6)
    assert O.inertial_power(ins, 0.3, "l") == 0.0 and O.inertial_power(ins, 0.3, "r") == 0.0

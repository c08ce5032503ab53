"""Pins of the oracle's free-flight system (Sec. 3.6, eq. oh_my_god_look_a_vector)
and of the aerodynamic power (eq. insect_power) against facts that do not come
from the oracle's own formulas: the yaw-pitch-roll matrix of Sec. 3.1, an
independent RK4 integration, closed forms (free fall, torque-free precession of
an axisymmetric top), conservation laws (angular momentum and energy of a
torque-free body, total momentum of fluid plus solid) and the equivalence of
the power with the work rate of the penalization force."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _rot_err(A, B):
    return float(np.max(np.abs(np.asarray(A) - np.asarray(B))))


def test_quaternion_matrix_reproduces_yaw_pitch_roll():
    rng = np.random.default_rng(7)
    for _ in range(20):
        psi, beta, gamma = rng.uniform(-math.pi, math.pi, 3)
        ins = O.Insect(psi=psi, beta=beta, gamma=gamma)
        eps = O.quaternion_from_angles(psi, beta, gamma)
        assert abs(np.sum(eps ** 2) - 1.0) < 1e-15
        # M_body of the quaternion equals Rx(psi) Ry(beta) Rz(gamma) of Sec. 3.1
        assert _rot_err(O.M_body_of_quaternion(eps), O.M_body(ins, 0.0)) < 1e-14
        Q = O.quaternion_matrix(eps)
        assert _rot_err(Q @ Q.T, np.eye(3)) < 1e-14 and abs(np.linalg.det(Q) - 1.0) < 1e-14
    # a quarter turn about z: the printed matrix maps body x to global y
    Q = O.quaternion_matrix([math.cos(math.pi / 4), 0.0, 0.0, math.sin(math.pi / 4)])
    assert _rot_err(Q @ [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]) < 1e-15


def test_quaternion_rows_follow_the_prescribed_rotation():
    """eps' = 1/2 S^T Omega^(b) with Omega^(b) of the prescribed body angles
    (Sec. 3.1) must carry the quaternion along M_body(t): integrated by RK4."""
    ins = O.Insect(psi=0.2, beta=-0.4, gamma=0.7, psi_dot=1.3, beta_dot=-0.8, gamma_dot=0.5)

    def deps(t, e):
        y = np.zeros(13)
        y[6:10] = e
        y[10:13] = O.omega_body_b(ins, t)
        return O.solid_rhs(ins, y, np.zeros(3), np.zeros(3))[6:10]

    e = O.quaternion_from_angles(ins.psi, ins.beta, ins.gamma)
    t, dt = 0.0, 2e-3
    for _ in range(500):
        k1 = deps(t, e)
        k2 = deps(t + dt / 2, e + dt / 2 * k1)
        k3 = deps(t + dt / 2, e + dt / 2 * k2)
        k4 = deps(t + dt, e + dt * k3)
        e = e + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        t += dt
    assert _rot_err(O.M_body_of_quaternion(e), O.M_body(ins, t)) < 1e-10
    assert abs(np.sum(e ** 2) - 1.0) < 1e-10


def test_free_fall_closed_form_with_variable_steps():
    """No fluid force: velocities are exact under AB2 (constant acceleration) and
    positions are exact after the first (Euler) step, which misses g dt0^2 / 2."""
    g = 9.81
    ins = O.Insect(free_flight=True, mass=2.0, gravity=g)
    y = np.zeros(13)
    y[0:3] = (1.0, 2.0, 3.0)
    y[3:6] = (0.3, -0.2, 1.0)
    y[6] = 1.0
    dts = [1e-2 * (1.0 + 0.5 * math.sin(k)) for k in range(40)]
    f, dtp, t = None, 0.0, 0.0
    for dt in dts:
        y, f = O.solid_step(ins, y, f, np.zeros(3), np.zeros(3), dt, dtp)
        dtp, t = dt, t + dt
    exact_x = np.array([1.0 + 0.3 * t, 2.0 - 0.2 * t, 3.0 + 1.0 * t - 0.5 * g * t * t + 0.5 * g * dts[0] ** 2])
    exact_u = np.array([0.3, -0.2, 1.0 - g * t])
    assert np.max(np.abs(y[0:3] - exact_x)) < 1e-13
    assert np.max(np.abs(y[3:6] - exact_u)) < 1e-13
    assert _rot_err(y[6:13], [1.0, 0, 0, 0, 0, 0, 0]) == 0.0


def test_axisymmetric_top_precesses_at_the_closed_form_rate():
    J1, J3 = 1.0, 2.5
    ins = O.Insect(free_flight=True, inertia=(J1, J1, J3))
    a, wz = 0.4, 1.5
    y = np.zeros(13)
    y[6] = 1.0
    y[10:13] = (a, 0.0, wz)
    lam = (J3 - J1) / J1 * wz
    T = 2.0

    def err(dt):
        yy, f = y.copy(), None
        for _ in range(int(round(T / dt))):
            yy, f = O.solid_step(ins, yy, f, np.zeros(3), np.zeros(3), dt, dt)
        assert yy[12] == wz
        return np.max(np.abs(yy[10:12] - [a * math.cos(lam * T), a * math.sin(lam * T)]))

    e1, e2 = err(2e-3), err(1e-3)
    # AB2 phase error (5/12) lam^3 dt^2 T a, and second order in dt
    assert e2 < 5e-6 and 3.6 < e1 / e2 < 4.4


def test_torque_free_body_keeps_angular_momentum_and_energy():
    """Asymmetric body, no torque: L^(g) = M_body^T J Omega^(b) and the
    kinetic energy are invariants; AB2 keeps them to O(dt^2)."""
    J = np.array([1.0, 2.0, 3.0])
    ins = O.Insect(free_flight=True, inertia=tuple(J))
    y = np.zeros(13)
    y[6:10] = O.quaternion_from_angles(0.3, -0.2, 0.9)
    y[10:13] = (1.0, 0.2, 0.3)

    def inv(y):
        Lg = O.M_body_of_quaternion(y[6:10]).T @ (J * y[10:13])
        return Lg, 0.5 * float(np.sum(J * y[10:13] ** 2))

    L0, E0 = inv(y)
    f, dt = None, 1e-4
    for _ in range(10000):
        y, f = O.solid_step(ins, y, f, np.zeros(3), np.zeros(3), dt, dt)
    L1, E1 = inv(y)
    assert np.max(np.abs(L1 - L0)) < 1e-6 * np.linalg.norm(L0)
    assert abs(E1 - E0) < 1e-6 * E0
    assert abs(np.sum(y[6:10] ** 2) - 1.0) < 1e-15
    # the body did turn: Omega^(b) moved away from its start
    assert np.max(np.abs(y[10:13] - [1.0, 0.2, 0.3])) > 0.05


def test_dof_switches_freeze_their_rows():
    ins = O.Insect(free_flight=True, mass=1.5, inertia=(1.0, 2.0, 3.0), gravity=1.0,
                   dof=(1.0, 0.0, 1.0, 0.0, 1.0, 0.0))
    y0 = np.zeros(13)
    y0[3:6] = (0.1, 0.2, 0.3)
    y0[6:10] = O.quaternion_from_angles(0.1, 0.2, 0.3)
    y0[10:13] = (0.4, 0.5, 0.6)
    y, f = y0.copy(), None
    for _ in range(5):
        y, f = O.solid_step(ins, y, f, np.array([1.0, 2.0, 3.0]), np.array([0.5, -0.5, 0.25]), 1e-2, 1e-2)
    assert y[4] == y0[4] and y[10] == y0[10] and y[12] == y0[12]
    assert y[3] != y0[3] and y[5] != y0[5] and y[11] != y0[11]


def _sphere_ff(L, **kw):
    d = W.sphere_body(L)
    d.update(free_flight=True, **kw)
    return O.Insect.from_dict(d)


def test_fluid_plus_solid_momentum_balance():
    """Free sphere in a periodic box with the mean flow free: the fluid's mean
    momentum changes by minus the penalization force and the body by plus the
    force, so M u_cntr + (fluid momentum) changes only by gravity and the
    unsteady correction, step by step with the AB2 weights."""
    n, L, eta = 24, 4.0, 1e-2
    vol = 4.0 / 3.0 * math.pi * 0.5 ** 3
    ins = _sphere_ff(L, u_cntr=(0.5, 0.0, 0.2), mass=2.0 * vol, gravity=1.0, dof=(1, 1, 1, 0, 0, 0))
    p = O.Params(n, L, 0.05, eta, O.MEAN_FREE)
    st = O.init_state(p, W.inflow_noise(n, L, seed=1, rms=1e-2, kmax=4.0) * 0.0)
    ctl = O.StepControl(cfl=0.1)

    def ptot(s, ysol):
        pf = np.real(s.uh[:, 0, 0, 0]) / n ** 3 * L ** 3
        return pf + ins.mass * ysol[3:6]

    ysol = O.solid_init(ins, 0.0)
    C_prev, I_prev, dt_prev = np.zeros(3), None, 0.0
    for k in range(8):
        P0 = ptot(st, ysol)
        new, d = O.step(p, st, ctl, ins)
        I_now = new.I_prev[:, :3].sum(axis=0)
        C = (I_now - I_prev) / dt_prev if I_prev is not None else np.zeros(3)
        dt = d["dt"]
        if k == 0:
            b1, b2 = 1.0, 0.0
        else:
            r = dt / dt_prev
            b1, b2 = 1.0 + 0.5 * r, -0.5 * r
        expect = dt * (b1 * C + b2 * C_prev) - ins.mass * ins.gravity * dt * np.array([0.0, 0.0, 1.0])
        got = ptot(new, new.solid) - P0
        assert np.max(np.abs(got - expect)) < 1e-11 * max(1.0, np.max(np.abs(P0))), k
        st, ysol, C_prev, I_prev, dt_prev = new, new.solid, C, I_now, dt
    # the body moved and was slowed by the fluid (drag opposes u_x)
    assert st.solid[0] > 2.0 and 0.0 < st.solid[3] < 0.5


def test_spinning_sphere_slows_about_its_own_axis():
    """A sphere spinning about a body axis in fluid at rest, its body frame
    turned by a quarter yaw: the fluid torque in the body frame opposes the
    spin, so the spin decays and keeps its direction (a transposed M_body in
    m^(b) = M_body m^(g) would turn the torque into a driving one)."""
    n, L = 24, 4.0
    ins = _sphere_ff(L, gamma=math.pi / 2, inertia=(2.0, 2.0, 2.0), dof=(0, 0, 0, 1, 1, 1))
    ins.smooth = "cos"
    p = O.Params(n, L, 0.05, 1e-2, O.MEAN_FIXED)
    st = O.init_state(p, np.zeros((3, n, n, n)))
    y0 = O.solid_init(ins, 0.0)
    y0[10:13] = (2.0, 0.0, 0.0)
    st.solid = y0
    ctl = O.StepControl(cfl=0.1, dt_max=2e-3)
    spin = [2.0]
    for _ in range(10):
        st, d = O.step(p, st, ctl, ins)
        spin.append(float(np.linalg.norm(st.solid[10:13])))
    assert all(b < a for a, b in zip(spin, spin[1:]))
    om = st.solid[10:13]
    assert abs(om[1]) + abs(om[2]) < 1e-3 * abs(om[0])


def test_torque_about_the_centre_transfers_from_the_parts():
    """First step (no unsteady terms): the free-flight torque about x_cntr equals
    the sum of the part torques about their own reference points moved to
    x_cntr, m_c + (x_ref,c - x_cntr) x F_c."""
    n, L = 32, 4.0
    d = W.model_insect(n, L)
    d.update(free_flight=True, mass=0.1, inertia=(0.01, 0.01, 0.01))
    ins = O.Insect.from_dict(d)
    p = O.Params(n, L, 1 / 136, 5e-4, O.MEAN_FIXED)
    st = O.init_state(p, W.inflow_noise(n, L, seed=2, rms=1e-2, kmax=6.0))
    _, dg = O.step(p, st, O.StepControl(cfl=0.1), ins)
    xref = O.reference_points(ins, 0.0, O.solid_pose(O.solid_init(ins, 0.0)))
    xc = xref[0]
    m = sum(dg["M"][c] + np.cross(xref[c] - xc, dg["F"][c]) for c in range(3))
    assert np.max(np.abs(m - dg["m_cntr"])) < 1e-12 * np.max(np.abs(dg["m_cntr"]))
    assert np.max(np.abs(dg["F_total"] - dg["F"].sum(axis=0))) == 0.0
    assert np.max(np.abs(dg["pose"] - O.solid_init(ins, 0.0))) == 0.0


def test_aero_power_is_the_work_rate_of_the_penalization_force():
    """P_aero = -m . (Omega_w - Omega_b) equals minus the work rate of the
    penalization force on the wing's velocity relative to the body,
    -sum (u_s - u_b) . chi (u - u_s)/C_eta dV over the wing (first step: no
    unsteady terms); checked with a turned, rotating body."""
    n, L, eta = 32, 4.0, 5e-4
    d = W.model_insect(n, L)
    d.update(psi=0.2, beta=-0.3, gamma=0.4, psi_dot=0.5, gamma_dot=-0.3)
    ins = O.Insect.from_dict(d)
    g = O.Grid(n, L)
    p = O.Params(n, L, 1 / 136, eta, O.MEAN_FIXED)
    u0 = W.inflow_noise(n, L, seed=3, rms=1e-2, kmax=6.0)
    st = O.init_state(p, u0)
    t = 0.13
    st.t = t
    _, dg = O.step(p, st, O.StepControl(cfl=0.1), ins)
    u = O.velocity(p, st)
    chi, us, col = O.insect_mask(g, ins, t)
    xb = O.to_body(ins, t, np.stack(g.coords()))
    ub = O.body_velocity(ins, t, xb)
    for k, side in enumerate(("l", "r")):
        sel = col == 2 + k
        urel = O.wing_velocity(ins, t, side, xb)[:, sel] - ub[:, sel]
        fpen = chi[sel] * (u[:, sel] - us[:, sel]) / eta * g.dV
        P = -float(np.sum(urel * fpen))
        assert abs(P) > 1e-6
        assert abs(dg["P_aero"][k] - P) < 1e-11 * abs(P), side

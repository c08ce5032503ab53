"""Pins of the oracle's insect model, mask and force integrals (CPU only).

P9 force of a uniform flow, P10 mask volumes, P11 solid velocity against a
finite difference of the frame transforms, P12 left/right mirror symmetry,
P13 rotation matrices, P14 K values printed in the paper."""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.mark.parametrize("R", [O.Rx, O.Ry, O.Rz])
def test_rotation_matrices_are_proper_and_transpose_is_inverse_angle(R):
    for a in (0.3, -1.1, 2.7):
        M = R(a)
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-15)
        assert np.linalg.det(M) == pytest.approx(1.0, abs=1e-15)
        assert np.allclose(M.T, R(-a), atol=1e-16)


def test_passive_rotation_convention():
    # Rz(pi/2) maps the global x-axis onto -y of the rotated frame (passive form)
    assert np.allclose(O.Rz(math.pi / 2) @ [1, 0, 0], [0, -1, 0], atol=1e-16)
    assert np.allclose(O.Rx(math.pi / 2) @ [0, 1, 0], [0, 0, -1], atol=1e-16)
    assert np.allclose(O.Ry(math.pi / 2) @ [0, 0, 1], [-1, 0, 0], atol=1e-16)


def test_penalization_K_matches_printed_values(golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "penalization_K.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 6
    for name, L, n, eta, nu_expr, K, digits in rows:
        nu = eval(nu_expr, {"pi": math.pi})
        k = O.penalization_K(nu, float(eta), float(L) / int(n))
        assert round(k, int(digits)) == pytest.approx(float(K), abs=1e-12), name


def _insect(n=64, L=4.0, t=0.13):
    ins = O.Insect.from_dict(W.model_insect(n, L))
    return ins


def test_solid_velocity_is_time_derivative_of_material_point():
    # a point fixed in the wing frame moves as x_g(t) = x_c + M_body^T (pivot + M_stroke^T M_wing^T p)
    ins = O.Insect.from_dict(dict(W.model_insect(64, 4.0), theta=(0.1, 0.2, 0.3),
                                  psi=0.2, beta=-0.5, gamma=0.4,
                                  psi_dot=0.7, beta_dot=-0.3, gamma_dot=0.5,
                                  u_cntr=(0.1, -0.2, 0.05)))
    p = np.array([0.05, 0.6, 0.01])
    h = 1e-5

    def xg(t, side):
        piv = np.array(ins.pivot_l if side == "l" else ins.pivot_r)
        Mb = O.M_body(ins, t)
        xb = piv + O.M_stroke(ins, side).T @ O.M_wing(ins, t, side).T @ p
        return np.array(ins.x_cntr) + np.array(ins.u_cntr) * t + Mb.T @ xb

    for t in (0.0, 0.13, 0.61):
        for side in ("l", "r"):
            fd = (xg(t + h, side) - xg(t - h, side)) / (2 * h)
            xb = O.M_body(ins, t) @ (xg(t, side) - np.array(ins.x_cntr) - np.array(ins.u_cntr) * t)
            us = O.wing_velocity(ins, t, side, xb.reshape(3, 1))[:, 0]
            assert np.allclose(us, fd, atol=1e-8), (t, side, us, fd)


def test_body_velocity_is_time_derivative_of_material_point():
    ins = O.Insect.from_dict(dict(body="ellipsoid", x_cntr=(1.0, 1.0, 1.0), psi=0.3, beta=0.2,
                                  gamma=-0.4, psi_dot=0.9, beta_dot=0.4, gamma_dot=-0.6))
    pb = np.array([0.3, -0.1, 0.2])
    h = 1e-5
    xg = lambda t: np.array(ins.x_cntr) + O.M_body(ins, t).T @ pb
    for t in (0.0, 0.5):
        fd = (xg(t + h) - xg(t - h)) / (2 * h)
        ub = O.body_velocity(ins, t, pb.reshape(3, 1))[:, 0]
        assert np.allclose(ub, fd, atol=1e-8)


def test_wing_kinematics_convention():
    ins = _insect()
    phi, alpha, theta, dphi, dalpha, dtheta = O.wing_angles(ins, 0.0)
    assert phi == pytest.approx(70 * math.pi / 180) and alpha == pytest.approx(0, abs=1e-15)
    phi, alpha, *_ = O.wing_angles(ins, 0.25)
    assert phi == pytest.approx(0, abs=1e-15) and alpha == pytest.approx(45 * math.pi / 180)


def test_stroke_plane_is_horizontal_for_model_insect():
    # body pitch -45 deg and stroke-plane angle -45 deg: the flapping axis x_s is vertical
    ins = _insect()
    Ms = O.M_stroke(ins, "l") @ O.M_body(ins, 0.0)
    assert np.allclose(Ms[0], [0, 0, 1], atol=1e-15)


@pytest.mark.parametrize("smooth", ["cos", "tanh"])
def test_sphere_volume_converges(smooth):
    R = 0.5
    exact = 4.0 / 3.0 * math.pi * R ** 3
    errs = []
    for n in (32, 64, 128):
        g = O.Grid(n, 2.0)
        ins = O.Insect(body="sphere", x_cntr=(1.0, 1.0, 1.0), radius=R, smooth=smooth)
        chi, us, col = O.insect_mask(g, ins, 0.0)
        assert chi.min() >= 0.0 and chi.max() <= 1.0
        errs.append(abs(chi.sum() * g.dV - exact) / exact)
    # the smoothing layer is symmetric about delta = 0: O(h^2) volume error
    assert errs[2] < 5e-3
    assert errs[1] / errs[2] > 3.0


def test_ellipsoid_and_wing_volumes():
    n, L = 128, 1.4
    g = O.Grid(n, L)
    ins = O.Insect(body="ellipsoid", x_cntr=(0.7, 0.7, 0.7), a=0.5, b=0.1, beta=0.3, gamma=0.2)
    chi, _, _ = O.insect_mask(g, ins, 0.0)
    exact = 4.0 / 3.0 * math.pi * 0.5 * 0.1 ** 2
    assert abs(chi.sum() * g.dV - exact) / exact < 2e-2
    assert chi[n // 2, n // 2, n // 2] == 1.0 and chi[0, 0, 0] == 0.0
    # a single flat wing (thickness 0.1) lying in the wing frame
    ins = O.Insect(body="none", x_cntr=(0.7, 0.7, 0.7), wings=True, pivot_l=(0.0, -0.5, 0.0),
                   pivot_r=(0.0, -10.0, 0.0), wing_A=0.175, wing_B=0.5, wing_t=0.1)
    chi, us, col = O.insect_mask(g, ins, 0.0)
    exact = math.pi * 0.175 * 0.5 * 0.1
    assert abs(chi.sum() * g.dV - exact) / exact < 2e-2
    assert set(np.unique(col)) <= {0, 2}


def test_colours_and_argmax_parts():
    g = O.Grid(64, 4.0)
    ins = _insect(64)
    chi, us, col = O.insect_mask(g, ins, 0.1)
    vals = set(np.unique(col).tolist())
    assert vals == {0, 1, 2, 3}
    assert np.all(chi[col == 0] == 0.0) and np.all(chi[col > 0] > 0.0)
    assert np.all(us[:, col == 0] == 0.0)
    # body is tethered and not rotating: u_s = 0 on body points
    assert np.all(us[:, col == 1] == 0.0)


def test_uniform_flow_force_and_comoving_body():
    n = 32
    L = 4.0
    eta = 1e-2
    p = O.Params(n, L, 0.01, eta, O.MEAN_FIXED)
    g = O.Grid(n, L)
    U = np.array([0.7, -0.2, 0.1])
    u0 = np.ones((3, n, n, n)) * U[:, None, None, None]
    ins = O.Insect(body="sphere", x_cntr=(2.0, 2.0, 2.0), radius=0.6, smooth="cos")
    st = O.init_state(p, u0)
    _, d = O.step(p, st, O.StepControl(cfl=0.1), ins)
    chi, _, _ = O.insect_mask(g, ins, 0.0)
    vol = chi.sum() * g.dV
    assert np.allclose(d["F"][0], U * vol / eta, rtol=1e-12)
    # torque of a uniform load about the sphere centre vanishes (symmetric mask)
    assert np.max(np.abs(d["M"][0])) < 1e-10 * np.max(np.abs(d["F"][0]))
    # a body translating with the fluid feels no penalization force
    ins2 = O.Insect(body="sphere", x_cntr=(2.0, 2.0, 2.0), radius=0.6, smooth="cos", u_cntr=tuple(U))
    _, d2 = O.step(p, st, O.StepControl(cfl=0.1), ins2)
    assert np.max(np.abs(d2["F"][0])) < 1e-10 * np.max(np.abs(d["F"][0]))


def test_model_insect_mirror_symmetry():
    # at 96^3 the two wings' smoothing layers stay clear of the mid-plane y = L/2,
    # so no grid point has a left/right tie in the argmax of chi
    n = 96
    L = 4.0
    wl = W.WORKLOADS["insect256"]
    p = O.Params(n, L, wl["nu"], wl["eta"], O.MEAN_FIXED)
    ins = O.Insect.from_dict(W.model_insect(n, L))
    u0 = np.zeros((3, n, n, n))
    st, hist = O.run(p, u0, 2, O.StepControl(cfl=0.1, dt_max=1e-3), ins)
    for d in hist:
        F, M = d["F"], d["M"]
        scale = np.max(np.abs(F))
        assert scale > 0
        assert abs(F[:, 1].sum()) <= 1e-12 * scale
        # left and right wing forces are mirror images across y = L/2
        assert np.allclose(F[1] * [1, -1, 1], F[2], atol=1e-12 * scale)
    u = O.velocity(p, st)
    mirrored = u[:, :, (-np.arange(n)) % n, :] * np.array([1, -1, 1])[:, None, None, None]
    assert np.max(np.abs(mirrored - u)) <= 1e-12 * np.max(np.abs(u))


def test_part_choice_ties_go_to_the_lowest_colour():
    # a later part wins only by more than the relative tie tolerance
    st = np.array([[1.0, 1.0, 0.0, 0.0, 0.2],
                   [1.0 + 1e-12, 1.0 + 1e-6, 0.0, 0.0, 0.2 * (1 + 1e-10)],
                   [0.5, 0.5, 0.0, 1e-3, 0.2 * (1 - 1e-10)]])
    assert O.part_of_max(st).tolist() == [0, 1, 0, 2, 0]


def test_mirror_plane_points_take_the_left_wing():
    # at 48^3 the wing roots reach the mid-plane y = L/2 (a grid plane): both
    # wings give the same chi there up to rounding, so colour 2 (left) and the
    # left wing velocity must be chosen
    n, L = 48, 4.0
    g = O.Grid(n, L)
    ins = O.Insect.from_dict(W.model_insect(n, L))
    t = 0.1
    chi, us, col = O.insect_mask(g, ins, t)
    x, y, z = g.coords()
    xb = O.to_body(ins, t, np.stack([x, y, z]))
    wl = [O.chi_of_delta(O.delta_elliptic_wing(*O.wing_frame(ins, t, s, xb), ins.wing_A, ins.wing_B, ins.wing_t),
                         ins, g.dx) for s in ("l", "r")]
    j = n // 2
    both = (wl[0][:, j, :] > 1e-6) & (wl[1][:, j, :] > 1e-6)
    assert both.sum() > 0
    assert np.allclose(wl[0][:, j, :][both], wl[1][:, j, :][both], rtol=1e-12, atol=0)
    wing_pts = both & (col[:, j, :] > 1)
    assert wing_pts.sum() > 0 and np.all(col[:, j, :][wing_pts] == 2)
    ul = O.wing_velocity(ins, t, "l", xb)
    assert np.allclose(us[:, :, j, :][:, wing_pts], ul[:, :, j, :][:, wing_pts], rtol=0, atol=1e-14)


def test_pointwise_mask_equals_the_grid_mask():
    n, L = 32, 4.0
    g = O.Grid(n, L)
    ins = O.Insect.from_dict(W.model_insect(n, L))
    chi, us, col = O.insect_mask(g, ins, 0.2)
    rng = np.random.default_rng(0)
    idx = rng.integers(0, n, size=(3, 500))
    x, y, z = (idx[2] * g.dx, idx[1] * g.dx, idx[0] * g.dx)
    c2, u2, k2 = O.mask_at(ins, 0.2, g.dx, x, y, z)
    assert np.array_equal(c2, chi[idx[0], idx[1], idx[2]])
    assert np.array_equal(u2, us[:, idx[0], idx[1], idx[2]])
    assert np.array_equal(k2, col[idx[0], idx[1], idx[2]])

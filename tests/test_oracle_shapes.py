"""Pins of the oracle's general wing kinematics (Fourier and Hermite series,
Sec. 3.3), the polar-radius Fourier wing with its 25 000-sample table (Sec. 3.4,
eq. Fourier_radious_wing) and the multi-part body (Sec. 3.2): against the
sinusoidal kinematics, finite differences, interpolation error bounds and
orders, the polar area formula, exact circle distances, orientation and
mirror symmetry."""
import math

import numpy as np

import oracle as O
import workloads as W


def test_fourier_angles_reproduce_the_sinusoid():
    mean, amp, ph, f = 0.1, 1.2, 0.7, 1.3
    sine = O.Insect(freq=f, phi=(mean, amp, ph), alpha=(0.0, 0.5, -1.0), theta=(0.2, 0.1, 0.3))

    def coefs(m, a, p):
        return ((2 * m, a * math.cos(p)), (0.0, -a * math.sin(p)))

    four = O.Insect(freq=f, kin="fourier", kin_phi=coefs(mean, amp, ph), kin_alpha=coefs(0.0, 0.5, -1.0),
                    kin_theta=coefs(0.2, 0.1, 0.3))
    for t in np.linspace(0.0, 2.0, 17):
        assert np.allclose(O.wing_angles(sine, t), O.wing_angles(four, t), rtol=0, atol=1e-13)


def test_series_rates_are_time_derivatives():
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=6), rng.normal(size=6)
    vals, rates = rng.normal(size=8), rng.normal(size=8)
    for kin, c in (("fourier", (tuple(a), tuple(b))), ("hermite", (tuple(vals), tuple(rates)))):
        ins = O.Insect(freq=0.8, kin=kin, kin_phi=c, kin_alpha=c, kin_theta=c)
        h = 1e-6
        for t in rng.uniform(0.0, 3.0, 10):
            p0, *_ = O.wing_angles(ins, t - h)
            p1, *_ = O.wing_angles(ins, t + h)
            _, _, _, dphi, _, _ = O.wing_angles(ins, t)
            assert abs((p1 - p0) / (2 * h) - dphi) < 1e-6 * max(1.0, abs(dphi)), kin


def test_hermite_interpolates_nodes_and_converges_at_fourth_order():
    f = 1.0
    g = lambda t: 0.4 * math.sin(2 * math.pi * t) + 0.2 * math.cos(6 * math.pi * t)
    dg = lambda t: 0.8 * math.pi * math.cos(2 * math.pi * t) - 1.2 * math.pi * math.sin(6 * math.pi * t)

    def err(K):
        tj = np.arange(K) / K
        ins = O.Insect(freq=f, kin="hermite", kin_phi=([g(t) for t in tj], [dg(t) for t in tj]))
        ins.kin_alpha = ins.kin_theta = ins.kin_phi
        for t in tj:  # nodes: exact values and rates
            v, _, _, dv, _, _ = O.wing_angles(ins, t + 1.0)  # one period later
            assert abs(v - g(t)) < 1e-13 and abs(dv - dg(t)) < 1e-11
        ts = np.linspace(0.0, 1.0, 397)
        return max(abs(O.wing_angles(ins, t)[0] - g(t)) for t in ts)

    e1, e2 = err(16), err(32)
    assert e2 < 2e-4 and 12.0 < e1 / e2 < 20.0


def test_hermite_is_continuous_with_its_rate_across_nodes():
    rng = np.random.default_rng(5)
    vals, rates = rng.normal(size=6), rng.normal(size=6)
    ins = O.Insect(freq=2.0, kin="hermite", kin_phi=(tuple(vals), tuple(rates)))
    ins.kin_alpha = ins.kin_theta = ins.kin_phi
    h = 1.0 / (2.0 * 6)
    for j in range(7):
        t = j * h
        lo = O.wing_angles(ins, t - 1e-12)
        hi = O.wing_angles(ins, t + 1e-12)
        assert abs(lo[0] - hi[0]) < 1e-9 and abs(lo[3] - hi[3]) < 1e-8
        assert abs(hi[0] - vals[j % 6]) < 1e-9 and abs(hi[3] - rates[j % 6]) < 1e-8


def test_radius_table_interpolation_within_the_linear_bound():
    rng = np.random.default_rng(11)
    n = 12
    fa = np.concatenate([[0.6], 0.05 * rng.normal(size=n)])
    fb = np.concatenate([[0.0], 0.05 * rng.normal(size=n)])
    tab = O.wing_radius_table(fa, fb)
    assert tab.shape == (O.R_TABLE_SIZE,)
    v = rng.uniform(-1.0, 2.0, 5000)
    exact = O.wing_radius_series(fa, fb, v)
    got = O.wing_radius_lookup(tab, v)
    # |R''| <= sum (2 pi i)^2 (|a_i| + |b_i|); linear interpolation error <= dv^2/8 max|R''|
    r2 = sum((2 * math.pi * i) ** 2 * (abs(fa[i]) + abs(fb[i])) for i in range(1, n + 1))
    bound = (1.0 / O.R_TABLE_SIZE) ** 2 / 8.0 * r2
    assert np.max(np.abs(got - exact)) <= bound + 1e-15
    # at the nodes the table is the series itself
    j = rng.integers(0, O.R_TABLE_SIZE, 50)
    assert np.max(np.abs(O.wing_radius_lookup(tab, j / O.R_TABLE_SIZE) - tab[j])) < 1e-14


def test_circular_fourier_wing_is_the_exact_circle_distance():
    R0 = 0.3
    ins = O.Insect(wing_shape="fourier", wing_c=(0.05, 0.4), wing_fa=(2 * R0, 0.0), wing_fb=(0.0, 0.0), wing_t=0.02)
    tab = O.wing_radius_table(ins.wing_fa, ins.wing_fb)
    rng = np.random.default_rng(2)
    x, y = rng.uniform(-0.5, 0.6, 200), rng.uniform(-0.1, 0.9, 200)
    z = rng.uniform(-0.05, 0.05, 200)
    d = O.delta_fourier_wing(x, y, z, ins, tab)
    exact = np.maximum(np.abs(z) - 0.01, np.hypot(x - 0.05, y - 0.4) - R0)
    assert np.max(np.abs(d - exact)) < 1e-14


def test_fourier_wing_area_and_orientation():
    """In-plane area pi[(a_0/2)^2 + 1/2 sum (a_i^2 + b_i^2)] (the polar area
    integral by Parseval), and a b_1 term pushes the outline toward +y_w."""
    fa = (0.8, 0.04, 0.02, 0.0)
    fb = (0.0, 0.06, 0.0, -0.015)
    ins = O.Insect(wing_shape="fourier", wing_c=(0.0, 0.0), wing_fa=fa, wing_fb=fb, wing_t=1.0)
    tab = O.wing_radius_table(fa, fb)
    m = 1600
    g = (np.arange(m) + 0.5) / m * 1.2 - 0.6
    X, Y = np.meshgrid(g, g, indexing="ij")
    inside = O.delta_fourier_wing(X, Y, np.zeros_like(X), ins, tab) < 0.0
    area = inside.sum() * (1.2 / m) ** 2
    exact = math.pi * ((fa[0] / 2) ** 2 + 0.5 * sum(a * a + b * b for a, b in zip(fa[1:], fb[1:])))
    assert abs(area - exact) < 2e-3 * exact
    # R(1/4) = 0.4 + 0.06 - 0.015 (+y) and R(3/4) = 0.4 - 0.06 + 0.015 (-y)
    up = O.delta_fourier_wing(np.array([0.0]), np.array([0.44]), np.array([0.0]), ins, tab)[0]
    dn = O.delta_fourier_wing(np.array([0.0]), np.array([-0.44]), np.array([0.0]), ins, tab)[0]
    assert up < 0.0 < dn


def _fourier_insect(n, L=4.0):
    d = W.model_insect(n, L)
    d.update(wing_shape="fourier", wing_c=(0.02, 0.32),
             wing_fa=(0.42, 0.03, -0.02, 0.01), wing_fb=(0.0, 0.05, 0.015, -0.01))
    return O.Insect.from_dict(d)


def test_fourier_wing_insect_is_mirror_symmetric():
    n, L = 48, 4.0
    ins = _fourier_insect(n, L)
    g = O.Grid(n, L)
    chi, us, col = O.insect_mask(g, ins, 0.21)
    assert np.sum(col == 2) > 50 and np.sum(col == 3) > 50
    # y -> L - y: index j -> (n - j) mod n
    mir = lambda a: np.roll(a[:, ::-1, :], 1, axis=1)
    assert np.max(np.abs(chi - mir(chi))) < 1e-12
    swap = np.where(col == 2, 3, np.where(col == 3, 2, col))
    ok = chi > 1e-9
    assert np.array_equal(mir(swap)[ok], col[ok])
    assert np.max(np.abs(us[1] + mir(us[1]))) < 1e-12


def test_head_and_eyes_join_the_thorax():
    ins = O.Insect(body="ellipsoid", a=0.3, b=0.08, head_x=(0.32, 0.0, 0.0), head_r=0.07,
                   eye_x=(0.36, 0.05, 0.02), eye_r=0.03)
    pts = np.array([[0.0, 0.0, 0.0], [0.34, 0.0, 0.0], [0.37, 0.05, 0.02], [0.37, -0.05, 0.02],
                    [0.0, 0.3, 0.0], [0.39, 0.0, 0.0]]).T
    d = O.delta_body(ins, pts)
    thorax = O.delta_ellipsoid(pts[0], pts[1], pts[2], 0.3, 0.08)
    head = np.linalg.norm(pts - np.array([[0.32], [0.0], [0.0]]), axis=0) - 0.07
    assert np.all(d <= thorax + 1e-15) and np.all(d <= head + 1e-15)
    assert d[0] < 0 and d[1] < 0 and d[2] < 0 and d[3] < 0 and d[4] > 0
    # the head alone, far from the thorax, is the sphere distance
    far = O.Insect(body="ellipsoid", a=1e-3, b=1e-3, head_x=(0.5, 0.0, 0.0), head_r=0.1)
    q = np.array([[0.5, 0.05, 0.0], [0.65, 0.0, 0.0]]).T
    assert np.allclose(O.delta_body(far, q), [-0.05, 0.05], atol=1e-15)
    # the eyes are a mirrored pair
    e = O.delta_body(ins, np.array([[0.36, 0.05, 0.02], [0.36, -0.05, 0.02]]).T)
    assert abs(e[0] - e[1]) < 1e-15


def test_rectangular_wing_is_the_intersection_of_half_spaces():
    ins = O.Insect(wing_shape="rectangle", rect_a=0.16667, rect_tip=1.0, rect_b=0.0667, rect_B=0.4167,
                   wing_t=0.04171)
    B, b, a, tip = ins.rect_B, ins.rect_b, ins.rect_a, ins.rect_tip
    # centre: minus the smallest half-width (here the thickness)
    xm, ym = b - B / 2, (a + tip) / 2
    d0 = O.delta_rect_wing(np.array([xm]), np.array([ym]), np.array([0.0]), ins)[0]
    assert abs(d0 + min(B / 2, (tip - a) / 2, ins.wing_t / 2)) < 1e-15
    # outside along each axis through the centre: the distance to that face
    for x, y, dist in ((b + 0.1, ym, 0.1), (b - B - 0.05, ym, 0.05), (xm, tip + 0.2, 0.2), (xm, a - 0.03, 0.03)):
        assert abs(O.delta_rect_wing(np.array([x]), np.array([y]), np.array([0.0]), ins)[0] - dist) < 1e-14
    # in-plane area B (tip - a)
    m = 1200
    gx = (np.arange(m) + 0.5) / m * 0.6 - 0.4
    gy = (np.arange(m) + 0.5) / m * 1.2 - 0.1
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    inside = O.delta_rect_wing(X, Y, np.zeros_like(X), ins) < 0.0
    area = inside.sum() * (0.6 / m) * (1.2 / m)
    assert abs(area - B * (tip - a)) < 3e-3 * B * (tip - a)
    # the printed a = 1.6667 leaves an empty span below the unit tip
    bad = O.Insect(wing_shape="rectangle", rect_a=1.6667, rect_tip=1.0, rect_b=b, rect_B=B, wing_t=0.04171)
    assert np.all(O.delta_rect_wing(X, Y, np.zeros_like(X), bad) > 0.0)


def test_rectangular_wing_insect_is_mirror_symmetric():
    n, L = 48, 4.0
    d = W.model_insect(n, L)
    d.update(wing_shape="rectangle", rect_a=0.1, rect_tip=0.55, rect_b=0.06, rect_B=0.25)
    ins = O.Insect.from_dict(d)
    g = O.Grid(n, L)
    chi, us, col = O.insect_mask(g, ins, 0.29)
    assert np.sum(col == 2) > 50 and np.sum(col == 3) > 50
    mir = lambda a: np.roll(a[:, ::-1, :], 1, axis=1)
    assert np.max(np.abs(chi - mir(chi))) < 1e-12
    swap = np.where(col == 2, 3, np.where(col == 3, 2, col))
    ok = chi > 1e-9
    assert np.array_equal(mir(swap)[ok], col[ok])

"""General shapes and kinematics (Sec. 3.2-3.4) on the GPU against the FP64
oracle: Fourier-radius wings through the 25 000-sample table, head and eye
spheres, Fourier and Hermite wing angle series; table rebuilds in plans and
ensembles; parameter checks."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import paper_1506_06513_amd as F
import workloads as W

pytestmark = pytest.mark.gpu

L = 4.0


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def np_of(t):
    return t.detach().double().cpu().numpy()


def fourier_wing_insect(n, **kw):
    d = W.model_insect(n, L)
    d.update(wing_shape="fourier", wing_c=(0.02, 0.32),
             wing_fa=(0.42, 0.03, -0.02, 0.01, 0.004), wing_fb=(0.0, 0.05, 0.015, -0.01, 0.003),
             head_x=(0.52, 0.0, 0.02), head_r=0.08, eye_x=(0.56, 0.05, 0.05), eye_r=0.035)
    d.update(kw)
    return d


def fourier_kinematics(phi_m=70.0, alpha_m=45.0):
    r = math.radians
    # stroke: phi_m cos(2 pi f t) plus a second harmonic; feathering: sin-like with a third harmonic
    return dict(kin="fourier",
                kin_phi=((0.0, r(phi_m), r(4.0), 0.0), (0.0, 0.0, r(2.0), 0.0)),
                kin_alpha=((0.0, 0.0, 0.0, r(3.0)), (0.0, r(alpha_m), 0.0, r(-2.0))),
                kin_theta=((r(2.0), 0.0, r(3.0), 0.0), (0.0, r(1.0), 0.0, 0.0)))


def hermite_kinematics(K=12, phi_m=70.0, alpha_m=45.0):
    r = math.radians
    tj = np.arange(K) / K
    w = 2 * math.pi
    phi = (r(phi_m) * np.cos(w * tj), -r(phi_m) * w * np.sin(w * tj))
    alpha = (r(alpha_m) * np.sin(w * tj), r(alpha_m) * w * np.cos(w * tj))
    theta = (r(5.0) * np.sin(2 * w * tj), r(5.0) * 2 * w * np.cos(2 * w * tj))
    return dict(kin="hermite", kin_phi=tuple(map(tuple, phi)), kin_alpha=tuple(map(tuple, alpha)),
                kin_theta=tuple(map(tuple, theta)))


def _part_stack(ins, g, t):
    x, y, z = g.coords()
    xb = O.to_body(ins, t, np.stack([x, y, z]))
    chis = [O.chi_of_delta(O.delta_body(ins, xb), ins, g.dx)]
    tab = O.wing_radius_table(ins.wing_fa, ins.wing_fb) if ins.wing_shape == "fourier" else None
    for s in "lr":
        xw = O.wing_frame(ins, t, s, xb)
        if tab is not None:
            d = O.delta_fourier_wing(xw[0], xw[1], xw[2], ins, tab)
        elif ins.wing_shape == "rectangle":
            d = O.delta_rect_wing(xw[0], xw[1], xw[2], ins)
        else:
            d = O.delta_elliptic_wing(xw[0], xw[1], xw[2], ins.wing_A, ins.wing_B, ins.wing_t)
        chis.append(O.chi_of_delta(d, ins, g.dx))
    return np.stack(chis)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fourier_wing_and_head_mask_matches_oracle(dtype):
    n = 96
    d = fourier_wing_insect(n, **fourier_kinematics())
    ins = O.Insect.from_dict(d)
    g = O.Grid(n, L)
    P = F.Plan(n, L, 0.01, 1e-3, dtype)
    for t in (0.0, 0.17, 0.38):
        chi_o, us_o, col_o = O.insect_mask(g, ins, t)
        chi, us, col = P.mask(d, t)
        tol = 1e-13 if dtype == "f64" else 3e-5
        assert np.max(np.abs(np_of(chi) - chi_o)) <= tol
        st = np.sort(_part_stack(ins, g, t), axis=0)
        gap = 1e-9 if dtype == "f64" else 1e-5
        ok = ~((st[-1] > 0) & (np.abs(st[-1] - st[-2]) < gap)) & (chi_o > (1e-12 if dtype == "f64" else 1e-6))
        assert np.array_equal(np_of(col)[ok].astype(int), col_o[ok])
        assert np.max(np.abs(np_of(us)[:, ok] - us_o[:, ok])) <= (1e-12 if dtype == "f64" else 3e-5)
        # both wings and the head are present
        assert np.sum(col_o == 2) > 100 and np.sum(col_o == 3) > 100


def rect_wing_insect(n, **kw):
    d = W.model_insect(n, L)
    d.update(wing_shape="rectangle", rect_a=0.1, rect_tip=0.55, rect_b=0.06, rect_B=0.25)
    d.update(kw)
    return d


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rectangular_wing_mask_and_steps_match_oracle(dtype):
    n = 96
    d = rect_wing_insect(n)
    ins = O.Insect.from_dict(d)
    g = O.Grid(n, L)
    P = F.Plan(n, L, 0.01, 1e-3, dtype)
    for t in (0.0, 0.23):
        chi_o, us_o, col_o = O.insect_mask(g, ins, t)
        chi, us, col = P.mask(d, t)
        assert np.max(np.abs(np_of(chi) - chi_o)) <= (1e-13 if dtype == "f64" else 3e-5)
        st = np.sort(_part_stack(ins, g, t), axis=0)
        gap = 1e-9 if dtype == "f64" else 1e-5
        ok = ~((st[-1] > 0) & (np.abs(st[-1] - st[-2]) < gap)) & (chi_o > (1e-12 if dtype == "f64" else 1e-6))
        assert np.array_equal(np_of(col)[ok].astype(int), col_o[ok])
        assert np.sum(col_o == 2) > 100
    m, nu, eta, steps = 48, 1 / 136, 5e-4, 6
    body = rect_wing_insect(m)
    u0 = W.inflow_noise(m, L, seed=42, rms=1e-2, kmax=6.0)
    p = O.Params(m, L, nu, eta, O.MEAN_FIXED)
    ost, _ = O.run(p, u0, steps, O.StepControl(cfl=0.1), O.Insect.from_dict(body))
    Q = F.Plan(m, L, nu, eta, dtype)
    s = Q.new_state(torch.from_numpy(u0))
    Q.step(s, steps, body, cfl=0.1)
    assert rel_l2(Q.velocity(s).cpu().numpy(), O.velocity(p, ost)) < (1e-11 if dtype == "f64" else 2e-5)


@pytest.mark.parametrize("kin", ["fourier", "hermite"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_general_insect_steps_match_oracle(kin, dtype):
    n, nu, eta, steps = 48, 1 / 136, 5e-4, 8
    extra = fourier_kinematics() if kin == "fourier" else hermite_kinematics()
    body = fourier_wing_insect(n, **extra)
    u0 = W.inflow_noise(n, L, seed=40, rms=1e-2, kmax=6.0)
    p = O.Params(n, L, nu, eta, O.MEAN_FIXED)
    ost, oh = O.run(p, u0, steps, O.StepControl(cfl=0.1), O.Insect.from_dict(body))
    P = F.Plan(n, L, nu, eta, dtype)
    st = P.new_state(torch.from_numpy(u0))
    h = P.step(st, steps, body, history=True, cfl=0.1).cpu().numpy()
    assert rel_l2(P.velocity(st).cpu().numpy(), O.velocity(p, ost)) < (1e-11 if dtype == "f64" else 2e-5)
    if dtype == "f64":
        for c in range(3):
            oF = np.array([d["F"][c] for d in oh])
            assert np.max(np.abs(h[:, 4 + 6 * c:7 + 6 * c] - oF)) <= 1e-9 * max(1e-12, np.max(np.abs(oF))), c
        oP = np.array([d["P_aero"] for d in oh])
        assert np.max(np.abs(h[:, 35:37] - oP)) <= 1e-9 * np.max(np.abs(oP))


@pytest.mark.parametrize("kin", ["sine", "fourier", "hermite"])
def test_inertial_and_total_power_match_oracle(kin):
    """P_inert (Sec. 3.5) with a general wing tensor of inertia: the device
    differentiates the wing's angular velocity exactly from the angle series,
    the oracle by a central difference; P_total = max(P_inert + P_aero, 0)."""
    n, nu, eta, steps = 32, 1 / 136, 5e-4, 6
    extra = {"sine": {}, "fourier": fourier_kinematics(), "hermite": hermite_kinematics()}[kin]
    body = dict(W.model_insect(n, L), wing_J=(2.0e-3, 5.0e-4, 2.4e-3, 3.0e-4, -2.0e-4, 1.5e-4), **extra)
    u0 = W.inflow_noise(n, L, seed=41, rms=1e-2, kmax=4.0)
    p = O.Params(n, L, nu, eta, O.MEAN_FIXED)
    ost, oh = O.run(p, u0, steps, O.StepControl(cfl=0.1), O.Insect.from_dict(body))
    P = F.Plan(n, L, nu, eta, "f64")
    st = P.new_state(torch.from_numpy(u0))
    h = P.step(st, steps, body, history=True, cfl=0.1).cpu().numpy()
    # the Hermite cubic's second derivative jumps at its nodes; t = 0 is one,
    # where the oracle's central difference averages the two sides
    r = slice(1, None) if kin == "hermite" else slice(None)
    oI = np.array([d["P_inert"] for d in oh])[r]
    oT = np.array([d["P_total"] for d in oh])[r]
    assert np.max(np.abs(oI)) > 1e-4
    assert np.max(np.abs(h[r, 37:39] - oI)) <= 1e-7 * np.max(np.abs(oI))
    assert np.max(np.abs(h[r, 39:41] - oT)) <= 1e-7 * max(np.max(np.abs(oT)), np.max(np.abs(oI)))
    assert np.all(h[:, 39:41] >= 0.0)
    # without a tensor of inertia the inertial power is zero and P_total = max(P_aero, 0)
    body0 = dict(body, wing_J=(0.0,) * 6)
    st0 = P.new_state(torch.from_numpy(u0))
    h0 = P.step(st0, 2, body0, history=True, cfl=0.1).cpu().numpy()
    assert np.all(h0[:, 37:39] == 0.0)
    assert np.array_equal(h0[:, 39:41], np.maximum(h0[:, 35:37], 0.0))


def test_wing_table_follows_coefficient_changes_and_ensembles():
    """A plan stepped with wing A, then wing B, equals fresh plans (the table is
    rebuilt on the stream); ensemble members with different wings equal their
    solo runs bitwise."""
    n = 48
    A = fourier_wing_insect(n)
    B = fourier_wing_insect(n, wing_fa=(0.40, -0.02, 0.03), wing_fb=(0.0, 0.04, -0.01), head_r=0.0)
    u0 = W.inflow_noise(n, L, seed=41, rms=1e-2, kmax=6.0)
    P = F.Plan(n, L, 0.01, 1e-3, "f32")
    s1 = P.new_state(torch.from_numpy(u0))
    P.step(s1, 3, A, cfl=0.1)
    s2 = P.new_state(torch.from_numpy(u0))
    P.step(s2, 3, B, cfl=0.1)
    Q = F.Plan(n, L, 0.01, 1e-3, "f32")
    r2 = Q.new_state(torch.from_numpy(u0))
    Q.step(r2, 3, B, cfl=0.1)
    assert torch.equal(P.uhat(s2), Q.uhat(r2))
    R = F.Plan(n, L, 0.01, 1e-3, "f32")
    r1 = R.new_state(torch.from_numpy(u0))
    R.step(r1, 3, A, cfl=0.1)
    assert torch.equal(P.uhat(s1), R.uhat(r1))
    assert not torch.equal(P.uhat(s1), P.uhat(s2))

    specs = [(48, A), (48, B), (32, fourier_wing_insect(32, **hermite_kinematics())), (48, W.model_insect(48, L))]
    ens = F.Ensemble("f32")
    pairs = []
    for k, (m, body) in enumerate(specs):
        um = W.inflow_noise(m, L, seed=50 + k, rms=1e-2, kmax=6.0)
        Pa, Pb = F.Plan(m, L, 0.01, 1e-3, "f32"), F.Plan(m, L, 0.01, 1e-3, "f32")
        sa, sb = Pa.new_state(torch.from_numpy(um)), Pb.new_state(torch.from_numpy(um))
        ens.add(Pa, sa, body, cfl=0.1)
        pairs.append((Pa, sa, Pb, sb, body))
    ens.step(3, graph=True)
    for Pa, sa, Pb, sb, body in pairs:
        Pb.step(sb, 3, body, cfl=0.1)
    torch.cuda.synchronize()
    for i, (Pa, sa, Pb, sb, _) in enumerate(pairs):
        assert torch.equal(Pa.uhat(sa), Pb.uhat(sb)), i
    ens.close()


def test_invalid_shape_parameters_are_rejected():
    n = 32
    P = F.Plan(n, L, 0.01, 1e-3, "f32")
    st = P.new_state(torch.zeros((3, n, n, n)))
    bad = [fourier_wing_insect(n, head_r=-0.1)]
    h = hermite_kinematics(K=2)
    h["kin_phi"] = ((0.1,), (0.0,))
    h["kin_alpha"] = h["kin_theta"] = h["kin_phi"]
    bad.append(fourier_wing_insect(n, **h))  # one Hermite node
    for body in bad:
        with pytest.raises(F.FlusiError) as e:
            P.step(st, 1, body, cfl=0.1)
        assert e.value.code == F.FLUSI_EINVAL
    with pytest.raises(ValueError):
        F.make_insect(fourier_wing_insect(n, wing_fa=tuple([0.1] * 40), wing_fb=tuple([0.0] * 40)))
    assert P.time(st)[1] == 0

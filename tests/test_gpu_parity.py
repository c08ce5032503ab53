"""HIP library vs the FP64 oracle, element by element (needs an MI355X).

Tolerances: FP64 relative L2 <= 1e-11 after 100 steps, FP32 <= 2e-5 (the
stated targets); single transforms are held to tighter bounds derived from
the transform's rounding (about 1e-15 * log2 n for FP64, 1e-7 * log2 n for
FP32).  Integer tables are compared bit for bit."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

import paper_1506_06513_amd as F  # noqa: E402

FFT_TOL = {"f64": 1e-13, "f32": 3e-6}


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def np_of(t):
    return t.detach().cpu().numpy()


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [16, 24, 32, 48, 64, 96, 128])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fft_r2c_c2r_match_oracle(n, dtype):
    rng = np.random.default_rng(n)
    f = rng.standard_normal((2, n, n, n))
    P = F.Plan(n, 2 * math.pi, 0.0, 1.0, dtype)
    fh = P.r2c(torch.from_numpy(f))
    ref = O.r2c(f)
    assert rel_l2(np_of(fh), ref) < FFT_TOL[dtype]
    # inverse of a Hermitian spectrum returns the field; input is preserved
    keep = fh.clone()
    back = P.c2r(fh)
    assert rel_l2(np_of(back), f) < FFT_TOL[dtype]
    assert torch.equal(keep, fh)
    # inverse on the oracle's spectrum vs the oracle's inverse
    g = O.c2r(ref, n)
    assert rel_l2(np_of(P.c2r(torch.from_numpy(ref))), g) < FFT_TOL[dtype]


@pytest.mark.parametrize("n", [32, 96, 256])
def test_tables_are_bit_exact(n):
    P = F.Plan(n, 1.0, 0.0, 1.0, "f64")
    j, keep = F.flusi_tables(P.handle, n)
    assert np.array_equal(j, O.signed_index(n))
    assert np.array_equal(keep.astype(bool), O.dealias_keep(O.signed_index(n), n))


def _unambiguous(ins, g, t, gap=1e-9):
    """Grid points where the largest part chi is not within `gap` of the next."""
    x, y, z = g.coords()
    xb = O.to_body(ins, t, np.stack([x, y, z]))
    chis = [O.chi_of_delta(O.delta_ellipsoid(xb[0], xb[1], xb[2], ins.a, ins.b), ins, g.dx)
            if ins.body == "ellipsoid" else np.zeros(x.shape)]
    if ins.body == "sphere":
        chis = [O.chi_of_delta(np.sqrt((x - ins.x_cntr[0]) ** 2 + (y - ins.x_cntr[1]) ** 2
                                       + (z - ins.x_cntr[2]) ** 2) - ins.radius, ins, g.dx)]
    if ins.wings:
        for s in "lr":
            xw = O.wing_frame(ins, t, s, xb)
            chis.append(O.chi_of_delta(O.delta_elliptic_wing(xw[0], xw[1], xw[2], ins.wing_A, ins.wing_B,
                                                             ins.wing_t), ins, g.dx))
    st = np.sort(np.stack(chis), axis=0)
    if st.shape[0] == 1:
        return np.ones(x.shape, bool)
    return ~((st[-1] > 0) & (np.abs(st[-1] - st[-2]) < gap))


@pytest.mark.parametrize("case", ["sphere", "insect"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mask_matches_oracle(case, dtype):
    n, L = 96, 4.0
    d = W.sphere_body(L) if case == "sphere" else W.model_insect(n, L)
    ins = O.Insect.from_dict(d)
    g = O.Grid(n, L)
    for t in (0.0, 0.13, 0.41):
        chi_o, us_o, col_o = O.insect_mask(g, ins, t)
        P = F.Plan(n, L, 0.01, 1e-3, dtype)
        chi, us, col = P.mask(d, t)
        # FP32 geometry: lengths of order 1 carry ~1e-7 rounding, amplified by
        # the mask slope ~1/h across the smoothing layer
        tol = 1e-13 if dtype == "f64" else 3e-5
        assert np.max(np.abs(np_of(chi) - chi_o)) <= tol
        # colour and u_s are unique where one part clearly dominates and chi is not a
        # rounding-level tail value (0.5*(1 - tanh) far outside the body)
        # the FP32 path evaluates the geometry in FP32
        ok = _unambiguous(ins, g, t, 1e-9 if dtype == "f64" else 1e-5) & (chi_o > (1e-12 if dtype == "f64" else 1e-6))
        gc, gchi = np_of(col), np_of(chi)
        assert np.array_equal(gc[ok], col_o[ok])
        assert np.all(gc[gchi == 0] == 0)
        assert np.max(np.abs(np_of(us)[:, ok] - us_o[:, ok])) <= (tol * 10 if dtype == "f64" else 3e-5)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rhs_matches_oracle(dtype):
    n, L = 64, 4.0
    p = O.Params(n, L, 0.01, 1e-3, O.MEAN_FIXED)
    g = O.Grid(n, L)
    u0 = W.inflow_noise(n, L, seed=4, rms=0.3, kmax=12.0)
    uh = O.import_field(g, u0)
    ins = O.Insect.from_dict(W.sphere_body(L))
    chi, us, _ = O.insect_mask(g, ins, 0.0)
    ref, u = O.rhs_hat(p, g, uh, chi, us)
    P = F.Plan(n, L, p.nu, p.eta, dtype)
    got, umax = P.rhs(torch.from_numpy(uh), torch.from_numpy(chi), torch.from_numpy(us),
                      F.FLUSI_MEAN_FIXED, want_umax=True)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert rel_l2(np_of(got), ref) < tol
    assert umax == pytest.approx(O.umax_of(u), rel=1e-12 if dtype == "f64" else 1e-6)


@pytest.mark.parametrize("n", [32, 48, 96])
def test_state_import_and_export(n):
    L = 2 * math.pi
    u0 = W.random_bandlimited(n, 5, kmax=n / 2.5)
    g = O.Grid(n, L)
    ref_uh = O.import_field(g, u0)
    P = F.Plan(n, L, 0.01, 1.0, "f64")
    st = P.new_state(torch.from_numpy(u0))
    assert rel_l2(np_of(P.uhat(st)), ref_uh) < 1e-13
    assert rel_l2(np_of(P.velocity(st)), O.c2r(ref_uh, n)) < 1e-13
    assert P.time(st) == (0.0, 0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_taylor_green_32_100_steps(dtype):
    # 32^3, L = 2 pi, nu = 0.01, fixed dt = 1e-3, 100 steps: closed form exp(-2 nu t)
    wl = W.WORKLOADS["tg32"]
    n = wl["n"]
    u0 = W.taylor_green(n)
    P = F.Plan(n, wl["L"], wl["nu"], wl["eta"], dtype)
    st = P.new_state(torch.from_numpy(u0))
    hist = P.step(st, 100, None, dt_fixed=1e-3, mean_mode=F.FLUSI_MEAN_FREE, history=True)
    t, nst = P.time(st)
    assert nst == 100 and t == pytest.approx(0.1, abs=1e-14)
    u = np_of(P.velocity(st))
    exact = u0 * math.exp(-2 * wl["nu"] * t)
    p = O.Params(n, wl["L"], wl["nu"], wl["eta"], O.MEAN_FREE)
    ost, ohist = O.run(p, u0, 100, O.StepControl(dt_fixed=1e-3))
    ou = O.velocity(p, ost)
    tol = 1e-11 if dtype == "f64" else 2e-5
    assert rel_l2(u, ou) < tol
    assert rel_l2(u, exact) < tol
    h = np_of(hist)
    assert np.allclose(h[:, 0], [d["t"] for d in ohist], rtol=0, atol=1e-14)
    assert np.allclose(h[:, 3], [d["E"] for d in ohist], rtol=1e-11 if dtype == "f64" else 1e-5)


def _compare_run(n, L, nu, eta, insect, u0, steps, dtype, ctl_kw, gpu_kw):
    p = O.Params(n, L, nu, eta, O.MEAN_FIXED)
    ins = O.Insect.from_dict(insect) if insect else None
    ost, ohist = O.run(p, u0, steps, O.StepControl(**ctl_kw), ins)
    ou = O.velocity(p, ost)
    P = F.Plan(n, L, nu, eta, dtype)
    st = P.new_state(torch.from_numpy(u0))
    hist = np_of(P.step(st, steps, insect, history=True, **gpu_kw))
    u = np_of(P.velocity(st))
    rc, last = P.forces(st)
    assert rc == 0
    return ou, ohist, u, hist


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sphere_48_adaptive_20_steps(dtype):
    n, L = 48, 4.0
    u0 = W.inflow_noise(n, L, seed=0, rms=1e-3, kmax=8.0)
    ou, oh, u, h = _compare_run(n, L, 0.01, 1e-3, W.sphere_body(L), u0, 20, dtype,
                                dict(cfl=0.1, eta_cap=0.5), dict(cfl=0.1, eta_cap=0.5))
    tol = 1e-11 if dtype == "f64" else 2e-5
    assert rel_l2(u, ou) < tol
    assert rel_l2(u - u.mean(axis=(1, 2, 3), keepdims=True),
                  ou - ou.mean(axis=(1, 2, 3), keepdims=True)) < (1e-9 if dtype == "f64" else 2e-3)
    odt = np.array([d["dt"] for d in oh])
    assert np.allclose(h[:, 1], odt, rtol=1e-12 if dtype == "f64" else 1e-6)
    oF = np.array([d["F"][0] for d in oh])
    scale = np.max(np.abs(oF))
    assert np.max(np.abs(h[:, 4:7] - oF)) <= (1e-10 if dtype == "f64" else 1e-4) * scale
    assert np.all(h[:, 4] > 0)  # drag on the sphere points downstream


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_insect_96_adaptive_10_steps(dtype):
    n, L = 96, 4.0
    wl = W.WORKLOADS["insect256"]
    u0 = np.zeros((3, n, n, n))
    ou, oh, u, h = _compare_run(n, L, wl["nu"], wl["eta"], W.model_insect(n, L), u0, 10, dtype,
                                dict(cfl=0.1, eta_cap=0.5), dict(cfl=0.1, eta_cap=0.5))
    tol = 1e-11 if dtype == "f64" else 2e-5
    assert rel_l2(u, ou) < tol
    for c in range(3):
        oF = np.array([d["F"][c] for d in oh[1:]])
        oM = np.array([d["M"][c] for d in oh[1:]])
        sF, sM = np.max(np.abs(oF)), np.max(np.abs(oM))
        assert np.max(np.abs(h[1:, 4 + 6 * c:7 + 6 * c] - oF)) <= (1e-9 if dtype == "f64" else 1e-3) * sF
        assert np.max(np.abs(h[1:, 7 + 6 * c:10 + 6 * c] - oM)) <= (1e-9 if dtype == "f64" else 1e-3) * sM

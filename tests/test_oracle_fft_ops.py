"""Pins of the oracle's transforms and spectral operators (CPU only).

P1 brute-force DFT, P2 round trip + Parseval, P3 numpy cross-check,
P4 projection / curl, P15 2/3-rule cutoff."""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W


def brute_dft3(f):
    """O(n^6) definition of the forward DFT with exp(-2 pi i j.x/n) on a cube."""
    n = f.shape[0]
    idx = np.arange(n)
    out = np.zeros((n, n, n // 2 + 1), dtype=complex)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    for kz in range(n):
        for ky in range(n):
            for kx in range(n // 2 + 1):
                ph = np.exp(-2j * math.pi * (kx * x + ky * y + kz * z) / n)
                out[kz, ky, kx] = np.sum(f * ph)
    return out


@pytest.mark.parametrize("n", [4, 6, 8, 12])
def test_r2c_matches_brute_force_dft(n):
    rng = np.random.default_rng(n)
    f = rng.standard_normal((n, n, n))
    ref = brute_dft3(f)
    got = O.r2c(f)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)) * n


@pytest.mark.parametrize("n", [6, 12, 16])
def test_c2r_inverts_brute_force(n):
    rng = np.random.default_rng(100 + n)
    f = rng.standard_normal((n, n, n))
    back = O.c2r(brute_dft3(f), n)
    assert np.max(np.abs(back - f)) <= 1e-13


@pytest.mark.parametrize("n", [24, 32, 48])
def test_round_trip_and_parseval(n):
    rng = np.random.default_rng(7)
    u = rng.standard_normal((3, n, n, n))
    uh = O.r2c(u)
    assert np.max(np.abs(O.c2r(uh, n) - u)) < 1e-13
    g = O.Grid(n, 2.0)
    e_phys = 0.5 * float(np.sum(u * u)) * g.dV
    assert abs(O.energy_spectral(g, uh) - e_phys) <= 1e-13 * e_phys


def test_r2c_matches_numpy_pocketfft():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((2, 18, 18, 18))
    ref = np.fft.rfftn(f, axes=(1, 2, 3))
    assert np.max(np.abs(O.r2c(f) - ref)) < 1e-12


def test_wavenumber_tables():
    assert list(O.signed_index(8)) == [0, 1, 2, 3, -4, -3, -2, -1]
    assert list(O.half_index(8)) == [0, 1, 2, 3, 4]
    assert list(O.signed_index(6)) == [0, 1, 2, -3, -2, -1]


def test_dealias_cutoff_against_the_caption(golden_dir):
    # The caption's highest resolved |j| is n/3.  The reading used here (keep iff
    # 3|j| < n) keeps every |j| below it and drops |j| = n/3 itself, the one
    # mode where the literal caption and the alias-free rule part.
    rows = [l.split() for l in open(os.path.join(golden_dir, "dealias_cutoff.txt"))
            if l.strip() and not l.startswith("#")]
    for n, L, jcap in rows:
        n, jcap = int(n), int(jcap)
        assert 3 * jcap == n
        assert O.dealias_kmax(n) == jcap - 1
        assert O.dealias_keep(np.array([jcap - 1]), n)[0]
        assert not O.dealias_keep(np.array([jcap, -jcap]), n).any()


@pytest.mark.parametrize("n", [24, 48, 96, 192, 384, 768])
def test_readings_part_only_where_three_divides_n(n):
    # for these n the literal caption would also keep |j| = n/3
    assert n % 3 == 0 and O.dealias_kmax(n) == n // 3 - 1


@pytest.mark.parametrize("n", [32, 64, 96, 128, 192, 256, 512])
def test_dealias_kmax_is_floor_n_minus_one_third(n):
    # the largest integer j with 3j < n
    assert O.dealias_kmax(n) == (n - 1) // 3


def test_projection_is_divergence_free_and_idempotent():
    n = 24
    g = O.Grid(n, 2 * math.pi)
    rng = np.random.default_rng(11)
    fh = O.r2c(rng.standard_normal((3, n, n, n))) * g.dealias()
    ph = O.project(g, fh)
    kx, ky, kz = g.k_vectors(derivative=True)
    kdot = kx * ph[0] + ky * ph[1] + kz * ph[2]
    kmag = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    pmag = np.sqrt(np.sum(np.abs(ph) ** 2, axis=0))
    assert np.max(np.abs(kdot)) <= 1e-14 * np.max(kmag * pmag)
    assert np.max(np.abs(O.project(g, ph) - ph)) <= 1e-14 * np.max(np.abs(ph))
    # k = 0 untouched
    assert np.allclose(ph[:, 0, 0, 0], fh[:, 0, 0, 0])
    # a pure gradient is removed entirely
    phi = O.r2c(rng.standard_normal((n, n, n))) * g.dealias()
    grad = np.stack([1j * kx * phi, 1j * ky * phi, 1j * kz * phi])
    assert np.max(np.abs(O.project(g, grad))) <= 1e-13 * np.max(np.abs(grad))


def test_curl_of_single_modes_and_of_gradient():
    n = 16
    L = 2 * math.pi
    g = O.Grid(n, L)
    a = W.grid_axis(n, L)
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    # u = (0, sin 2x, 0) -> curl = (0, 0, 2 cos 2x)
    u = np.stack([0 * x, np.sin(2 * x), 0 * x])
    w = O.c2r(O.curl_hat(g, O.r2c(u)), n)
    assert np.max(np.abs(w - np.stack([0 * x, 0 * x, 2 * np.cos(2 * x)]))) < 1e-13
    # u = (sin 3z, 0, cos y) -> curl = (-sin y, 3 cos 3z, 0)
    u = np.stack([np.sin(3 * z), 0 * x, np.cos(y)])
    w = O.c2r(O.curl_hat(g, O.r2c(u)), n)
    assert np.max(np.abs(w - np.stack([-np.sin(y), 3 * np.cos(3 * z), 0 * x]))) < 1e-13
    # curl of a gradient vanishes
    rng = np.random.default_rng(5)
    phi = O.r2c(rng.standard_normal((n, n, n))) * g.dealias()
    kx, ky, kz = g.k_vectors(derivative=True)
    grad = np.stack([1j * kx * phi, 1j * ky * phi, 1j * kz * phi])
    assert np.max(np.abs(O.curl_hat(g, grad))) <= 1e-14 * np.max(np.abs(grad)) * n


def test_nyquist_has_no_derivative():
    n = 8
    g = O.Grid(n, 2 * math.pi)
    kx, ky, kz = g.k_vectors(derivative=True)
    assert kx[0, 0, n // 2] == 0.0 and ky[0, n // 2, 0] == 0.0 and kz[n // 2, 0, 0] == 0.0
    kx2 = g.k2()
    assert kx2[0, 0, n // 2] == pytest.approx((n / 2) ** 2)

"""The allocation-free inverse transform flusi_fft_c2r_noalloc against
flusi_fft_c2r through the C ABI (needs an MI355X): bit for bit on two calls
in a row, the second with a smaller input, both also within the transform
tolerance of the oracle's inverse; sizes above the fixed scratch are
refused with an error."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1506_06513_amd as F

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.name}", flush=True)
    yield
    torch.cuda.synchronize()


def _spectrum(P, nf, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nf,) + P.shape)
    return P.r2c(torch.from_numpy(f)), f


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_c2r_equals_c2r_on_two_calls(dtype):
    tol = 1e-13 if dtype == "f64" else 3e-6
    # first call: three 64^3 fields; second: one 32^3 field (smaller input)
    for n, nf, seed in ((64, 3, 1), (32, 1, 2)):
        P = F.Plan(n, 1.0, 0.0, 1.0, dtype)
        fh, f = _spectrum(P, nf, seed)
        keep = fh.clone()
        ref = P.real(nf)
        F.flusi_fft_c2r(P.handle, fh, ref, nf)
        got = P.real(nf)
        F.flusi_fft_c2r_noalloc(P.handle, fh, got, nf)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (n, nf)
        assert torch.equal(fh, keep)  # input preserved
        o = O.c2r(fh.cpu().numpy(), n)
        err = float(np.linalg.norm(got.cpu().numpy() - o) / np.linalg.norm(o))
        assert err < tol, (n, nf, err)
        assert float(np.linalg.norm(got.cpu().numpy() - f) / np.linalg.norm(f)) < tol


def test_noalloc_c2r_refuses_sizes_above_the_scratch():
    P = F.Plan(256, 1.0, 0.0, 1.0, "f32")
    fh = torch.zeros((1, 256, 256, 129), dtype=torch.complex64, device="cuda")
    out = P.real(1)
    with pytest.raises(F.FlusiError) as e:
        F.flusi_fft_c2r_noalloc(P.handle, fh, out, 1)
    assert e.value.code == F.FLUSI_EINVAL and "scratch" in str(e.value)
    with pytest.raises(F.FlusiError):
        F.flusi_fft_c2r_noalloc(P.handle, fh, out, 0)

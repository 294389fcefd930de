"""Fourier-domain sparsification (Sec. 2.4, Alg. 2.4/2.5) through the C ABI
against the float64 oracle: zeroth and first order, rectangular shapes, the
exact limits, full size on sampled outputs, and the rejected cases."""
import numpy as np
import pytest

from oracle import sfft as osf
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu


def _smooth(m, n, seed):
    """Rows with decaying spectra plus noise: a few frequencies dominate."""
    return f32(inputs.sinusoid_rows(m, n, np.random.default_rng(seed)))


@pytest.mark.parametrize("m,n,p,k", [(64, 64, 40, 6), (96, 128, 50, 9), (256, 256, 256, 16), (200, 512, 64, 33),
                                     (50, 300, 40, 7), (70, 700, 64, 12)])
def test_sfft_zeroth_parity(m, n, p, k):
    note(f"sfft zeroth m={m} n={n} p={p} k={k}")
    A = _smooth(m, n, m + n)
    B = f32(np.random.default_rng(p).standard_normal((n, p)))
    dec = osf.SFFTDecomp(A, k)
    c = ctx()
    d = c.decompose(gpu(A), "sfft", k)
    assert d.info()["nnz"] == int(dec.row_mask.sum())
    got = host(c.approx_matmul(d, gpu(B)))
    assert rel(got, osf.product(dec, B)) < TOL_F32


@pytest.mark.parametrize("m,n,p,k", [(64, 64, 64, 6), (128, 256, 96, 12), (256, 128, 256, 7), (60, 300, 70, 9)])
def test_sfft_first_order_parity(m, n, p, k):
    note(f"sfft first order m={m} n={n} p={p} k={k}")
    A = _smooth(m, n, 3 * m + n)
    B = _smooth(n, p, 5 * n + p)
    decA, decB = osf.SFFTDecomp(A, k), osf.SFFTDecomp(B, k)
    c = ctx()
    dA = c.decompose(gpu(A), "sfft", k)
    dB = c.decompose(gpu(B), "sfft", k)
    got = host(c.approx_matmul(dA, gpu(B), dB))
    want = osf.product(decA, B, decB)
    assert rel(got, want) < TOL_F32
    # the first-order identity M = AB - dA dB holds for the float64 result
    err = rel(got, A @ B)
    note(f"  error vs AB {err:.3e}")


def test_sfft_limits():
    n, p = 128, 64
    A = _smooth(n, n, 1)
    B = f32(np.random.default_rng(2).standard_normal((n, p)))
    c = ctx()
    full = c.decompose(gpu(A), "sfft", n)
    assert rel(host(c.approx_matmul(full, gpu(B))), A @ B) < TOL_F32
    fB = c.decompose(gpu(B), "sfft", n)
    assert rel(host(c.approx_matmul(full, gpu(B), fB)), A @ B) < TOL_F32
    zero = c.decompose(gpu(A), "sfft", 0)
    assert np.max(np.abs(host(c.approx_matmul(zero, gpu(B))))) == 0.0


def test_sfft_rejected_cases():
    from paper_2504_19308_amd import AmmError
    n = 64
    A = _smooth(n, n, 4)
    c = ctx()
    d = c.decompose(gpu(A), "sfft", 4)
    with pytest.raises(AmmError):
        c.approx_matmul(d, gpu(np.ones((n, 7))))             # odd column count
    dt = c.decompose(gpu(A), "tsvd", 4)
    with pytest.raises(AmmError):
        c.approx_matmul(d, gpu(A), dt)                       # mixed with another kind
    with pytest.raises(AmmError):
        c.decompose(gpu(np.ones((1, 1))), "sfft", 1)         # neither side in [2, 16384]


def test_sfft_first_order_full_size_sampled():
    """n = 4096, k = 32, first order: 24 x 24 sampled outputs against the
    oracle's per-row / per-column evaluation."""
    torch = torch_cuda()
    n, k = 4096, 32
    note(f"sfft full size n={n} k={k}")
    A = _smooth(n, n, 40)
    B = _smooth(n, n, 41)
    c = ctx()
    Ag, Bg = gpu(A), gpu(B)
    dA = c.decompose(Ag, "sfft", k)
    dB = c.decompose(Bg, "sfft", k)
    M = c.approx_matmul(dA, Bg, dB)
    rng = np.random.default_rng(inputs.seed_of(6, 1))
    rows = np.sort(rng.choice(n, 24, replace=False))
    cols = np.sort(rng.choice(n, 24, replace=False))
    got = M[torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
    want = osf.product_entries(A, B, k, rows, cols, True)
    assert rel(got, want) < TOL_F32

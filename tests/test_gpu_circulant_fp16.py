"""Float16 spectral products (spectral_fp16, n >= 1024), Alg. 2.3 step 5 with
half-precision multiplicands.

Sides that are powers of two round both factors of every list-times-spectrum
product to float16: the eigenvalue lists (scaled by a power of two) and each
tile's forward spectrum (scaled by a power of two per tile); the products are
summed in float32 and both transforms stay float32.  Rounding a complex value
to nearest float16 parts changes it by at most u16 |z| (u16 = 2^-11), so the
spectral sum of term t,  L_t(p) X(p - k_t),  moves by at most
(2 u16 + u16^2) |L_t(p) X(p - k_t)|, and by Parseval the product moves by at
most about 2 u16 sum_t ||term_t||_F, with term_t the product of the single
component t (computed by the oracle).  The tests check the float16 result
against the float64 oracle within that bound (plus the float32 bar), and that
the error is above the float32 bar (the half-precision path is in use).
Other sides (the fused chirp-convolution kernel) widen the float16 lists and
multiply in float32: bound u16 sum_t ||term_t||_F."""
import numpy as np
import pytest

from oracle import circulant as oc
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu

U16 = 2.0 ** -11


class _Lists:
    def __init__(self, n, S, L):
        self.n, self.S, self.L = n, np.asarray(S, dtype=np.int64), np.asarray(L)


def _pair_lists(n, K, rng, scale=1.0, singles=False):
    """K/2 pair classes {k, n-k} with random lists, L_{n-k}[p] = conj(L_k[-p])
    (a real operator); with singles also the self-paired frequencies 0 and
    n/2, whose lists satisfy L[p] = conj(L[-p])."""
    neg = (-np.arange(n)) % n
    ks = rng.choice(np.arange(1, n // 2), K // 2, replace=False)
    S, L = [], []
    for k in ks:
        v = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * scale
        S += [int(k), int(n - k)]
        L += [v, np.conj(v[neg])]
    if singles:
        for k in (0, n // 2):
            v = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * scale
            S.append(k)
            L.append(0.5 * (v + np.conj(v[neg])))
    order = np.argsort(S)
    return [S[i] for i in order], np.array(L)[order]


def _terms(n, S, L, B):
    return sum(np.linalg.norm(np.real(oc.apply_zeroth(_Lists(n, [k], L[t:t + 1]), B))) for t, k in enumerate(S))


def _randn(n, p, seed):
    torch = torch_cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randn((n, p), generator=g, device="cuda", dtype=torch.float32)


@pytest.mark.parametrize("n,K,p,singles", [(1024, 6, 48, False), (4096, 10, 40, True), (8192, 4, 36, False),
                                           (16384, 64, 24, False), (16384, 6, 28, True), (16384, 4, 26, True)])
def test_fp16_products_bound(n, K, p, singles):
    """Imported lists (any scale: these are 1e-5 of unit size, below the
    float16 normal range before scaling), float16 products on and off.
    n = 16384 with p a multiple of 4 runs the two-pairs-per-workgroup kernel
    (p = 28: seven tiles), other p the one-pair kernel; singles adds the
    self-paired frequencies 0 and n/2."""
    note(f"fp16 products n={n} K={K} p={p} singles={singles}")
    rng = np.random.default_rng(n + K)
    S, L = _pair_lists(n, K, rng, scale=1e-5, singles=singles)
    c = ctx()
    d = c.import_circulant(n, S, L)
    B = _randn(n, p, n + 3)
    Bh = host(B)
    want = np.real(oc.apply_zeroth(_Lists(n, S, L), Bh))
    assert rel(host(c.approx_matmul(d, B)), want) < TOL_F32
    d.set_spectral_fp16(True)
    assert d.info()["spectral_fp16"] == 1
    got = host(c.approx_matmul(d, B))
    bound = 2.0 * U16 * (1.0 + U16) * _terms(n, S, L, Bh) / np.linalg.norm(want) + TOL_F32
    err = rel(got, want)
    note(f"  err {err:.3e} bound {bound:.3e}")
    assert TOL_F32 < err < bound
    d.set_spectral_fp16(False)
    assert rel(host(c.approx_matmul(d, B)), want) < TOL_F32


def test_fp16_scaled_columns():
    """Columns of very different magnitude in one tile: each tile's spectrum
    shares one power-of-two scale, so a small column keeps the absolute error
    of the tile's largest; columns in separate tiles keep their own scale."""
    n, K = 4096, 8
    rng = np.random.default_rng(5)
    S, L = _pair_lists(n, K, rng)
    c = ctx()
    d = c.import_circulant(n, S, L).set_spectral_fp16(True)
    torch = torch_cuda()
    B = _randn(n, 64, 9)
    B[:, 32:] *= 1e-30     # a whole tile of tiny columns (8 packed columns per tile at n = 4096)
    B[:, 1] *= 1e6         # a large column inside the first tile
    Bh = host(B)
    got = host(c.approx_matmul(d, B))
    for cols in (slice(0, 8), slice(32, 64)):
        want = np.real(oc.apply_zeroth(_Lists(n, S, L), Bh[:, cols]))
        bound = 2.0 * U16 * (1.0 + U16) * _terms(n, S, L, Bh[:, cols]) / np.linalg.norm(want) + TOL_F32
        assert rel(got[:, cols], want) < bound
    assert torch.isfinite(torch.from_numpy(got)).all()


def test_fp16_first_order():
    """A tilde B + Delta A B tilde with both circulant handles in float16
    products; the first-order term runs the row kernel with the adjoint lists."""
    n = 2048
    from paper_2504_19308_amd import inputs
    rng = np.random.default_rng(77)
    A = f32(inputs.toeplitz_uniform(n, rng) + 0.05 * rng.standard_normal((n, n)))
    B = f32(inputs.toeplitz_uniform(n, rng) + 0.05 * rng.standard_normal((n, n)))
    c = ctx()
    dA = c.decompose(gpu(A), "circulant", 6, spectral_fp16=True)
    dB = c.decompose(gpu(B), "circulant", 4, spectral_fp16=True)
    decA, decB = oc.CirculantDecomp(A, 6), oc.CirculantDecomp(B, 4)
    assert list(dA.frequencies()) == list(decA.S) and list(dB.frequencies()) == list(decB.S)
    got = host(c.approx_matmul(dA, gpu(B), dB))
    zeroth = np.real(oc.apply_zeroth(decA, B))
    dAres = A - np.real(decA.truncated_dense())
    first = np.real(oc.apply_first_order_term(decB, dAres))
    want = zeroth + first
    tz = _terms(n, list(decA.S), decA.L, B)
    tf = sum(np.linalg.norm(np.real(oc.apply_first_order_term(_Lists(n, [k], decB.L[t:t + 1]), dAres)))
             for t, k in enumerate(decB.S))
    bound = 2.0 * U16 * (1.0 + U16) * (tz + tf) / np.linalg.norm(want) + TOL_F32
    err = rel(got, want)
    note(f"  first order err {err:.3e} bound {bound:.3e}")
    assert TOL_F32 < err < bound


@pytest.mark.parametrize("n,K", [(1024, 9), (4096, 32), (1500, 12)])
def test_fp16_general_operand_bound(n, K):
    note(f"fp16 general operand n={n} K={K}")
    from paper_2504_19308_amd import inputs
    rng = np.random.default_rng(n + K)
    A = f32(inputs.toeplitz_uniform(n, rng) + 0.05 * rng.standard_normal((n, n)))
    B = f32(rng.standard_normal((n, 40)))
    dec = oc.CirculantDecomp(A, K)
    c = ctx()
    d = c.decompose(gpu(A), "circulant", K, spectral_fp16=True)
    assert d.info()["spectral_fp16"] == 1
    assert list(d.frequencies()) == list(dec.S)
    got = host(c.approx_matmul(d, gpu(B)))
    want = np.real(oc.apply_zeroth(dec, B))
    # powers of two: lists and spectra rounded; the chirp kernel: lists only
    factor = 2.0 * (1.0 + U16) if (n & (n - 1)) == 0 else 1.0
    bound = factor * U16 * _terms(n, list(dec.S), dec.L, B) / np.linalg.norm(want) + TOL_F32
    err = rel(got, want)
    assert TOL_F32 < err < bound   # half-precision factors are in use, within their bound
    d32 = c.decompose(gpu(A), "circulant", K)
    assert rel(host(c.approx_matmul(d32, gpu(B))), want) < TOL_F32


def test_fp16_small_n_keeps_float32():
    n = 512
    rng = np.random.default_rng(3)
    from paper_2504_19308_amd import inputs
    A = f32(inputs.toeplitz_uniform(n, rng) + 0.05 * rng.standard_normal((n, n)))
    c = ctx()
    d = c.decompose(gpu(A), "circulant", 5, spectral_fp16=True)
    assert d.info()["spectral_fp16"] == 0
    B = f32(rng.standard_normal((n, 8)))
    assert rel(host(c.approx_matmul(d, gpu(B))), np.real(oc.apply_zeroth(oc.CirculantDecomp(A, 5), B))) < TOL_F32
    with pytest.raises(Exception):
        d.set_spectral_fp16(True)

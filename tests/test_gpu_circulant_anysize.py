"""Circulant decomposition and products for sides that are not powers of two
(the paper's own examples use n = 700): Bluestein's chirp convolution on the
device (float64 decomposition; products in one fused float32 kernel up to
n = 2048, float64 steps above), against the float64 oracle (any n)."""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import product as op
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel

pytestmark = pytest.mark.gpu


def _toeplitz(n, seed, noise=0.05):
    rng = np.random.default_rng(seed)
    return f32(inputs.toeplitz_uniform(n, rng) + noise * rng.standard_normal((n, n)))


@pytest.mark.parametrize("n,K,p", [(3, 1, 5), (12, 5, 7), (100, 9, 31), (700, 11, 64), (1000, 32, 100),
                                   (2047, 20, 3), (2049, 6, 9)])
def test_anysize_decompose_and_zeroth(n, K, p):
    note(f"circulant any size n={n} K={K} p={p}")
    A = _toeplitz(n, n + K)
    B = f32(np.random.default_rng(p).standard_normal((n, p)))
    dec = oc.CirculantDecomp(A, K)
    c = ctx()
    d = c.decompose(gpu(A), "circulant", K)
    assert list(d.frequencies()) == list(dec.S)
    E = d.energies()
    assert np.max(np.abs(E - dec.E)) <= 1e-10 * np.max(dec.E)
    assert abs(d.info()["norm_residual"] - dec.norm_residual()) <= 1e-9 * dec.norm_residual() + 1e-12
    got = host(c.approx_matmul(d, gpu(B)))
    assert rel(got, np.real(oc.apply_zeroth(dec, B))) < TOL_F32


@pytest.mark.parametrize("n,KA,KB", [(700, 7, 5), (384 + 3, 6, 10), (1531, 9, 4)])
def test_anysize_first_order(n, KA, KB):
    note(f"circulant any size first order n={n}")
    A, B = _toeplitz(n, 1), _toeplitz(n, 2)
    decA, decB = oc.CirculantDecomp(A, KA), oc.CirculantDecomp(B, KB)
    c = ctx()
    dA = c.decompose(gpu(A), "circulant", KA)
    dB = c.decompose(gpu(B), "circulant", KB)
    got = host(c.approx_matmul(dA, gpu(B), dB))
    assert rel(got, op.algorithm(decA, B, decB)) < TOL_F32
    # M1 = AB - dA dB
    dAm = A - np.real(decA.truncated_dense())
    dBm = B - np.real(decB.truncated_dense())
    assert rel(got, A @ B - dAm @ dBm) < TOL_F32


def test_anysize_full_expansion_and_blocks():
    """K = n reproduces AB at n = 700; a 700 x 300 operand runs as square blocks
    of side 300 (not a power of two)."""
    n = 700
    A = f32(np.random.default_rng(5).standard_normal((n, n)))
    B = f32(np.random.default_rng(6).standard_normal((n, 40)))
    c = ctx()
    d = c.decompose(gpu(A), "circulant", n)
    assert rel(host(c.approx_matmul(d, gpu(B))), A @ B) < TOL_F32
    R = f32(np.random.default_rng(7).standard_normal((700, 300)))
    Bb = f32(np.random.default_rng(8).standard_normal((300, 20)))
    dec = oc.BlockedCirculant(R, 9)
    db = c.decompose(gpu(R), "circulant", 9)
    assert db.info()["blocks"] == dec.nb
    assert rel(host(c.approx_matmul(db, gpu(Bb))), oc.apply_blocked(dec, Bb)) < TOL_F32


def test_anysize_mu_and_plan_rejection():
    from paper_2504_19308_amd import AmmError
    from oracle import estimators as oe
    n = 300
    A = _toeplitz(n, 9)
    dec = oc.CirculantDecomp(A, 5)
    c = ctx()
    d = c.decompose(gpu(A), "circulant", 5)
    assert abs(d.info()["mu"] - oe.cd_mu(dec)) <= 1e-9 * oe.cd_mu(dec)
    B = gpu(np.ones((n, 8)))
    with pytest.raises(AmmError):
        c.batch_plan([d], [B])

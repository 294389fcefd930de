"""Circulant decomposition and products for sides that are not powers of two
(the paper's own examples use n = 700): Bluestein's chirp convolution on the
device (float64 decomposition; products in one fused float32 kernel up to
n = 2048, float64 steps above), against the float64 oracle (any n)."""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import product as op
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel, torch_cuda

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


def test_anysize_mu():
    from oracle import estimators as oe
    n = 300
    A = _toeplitz(n, 9)
    dec = oc.CirculantDecomp(A, 5)
    c = ctx()
    d = c.decompose(gpu(A), "circulant", 5)
    assert abs(d.info()["mu"] - oe.cd_mu(dec)) <= 1e-9 * oe.cd_mu(dec)


def test_anysize_batch_plan():
    """Plans take sides up to 2048 that are not powers of two (the fused
    kernel; square and blocked entries mixed with a power of two); graph
    replays equal the eager run and the oracle; a side of 2049 is rejected."""
    from paper_2504_19308_amd import AmmError
    torch = torch_cuda()
    c = ctx()
    cases = [(300, 300, 5, 24), (700, 300, 4, 9), (256, 256, 6, 16), (1000, 1000, 9, 31)]
    decs, Bs, wants = [], [], []
    for i, (m, n, K, p) in enumerate(cases):
        rng = np.random.default_rng(80 + i)
        A = f32(inputs.toeplitz_uniform(max(m, n), rng)[:m, :n] + 0.05 * rng.standard_normal((m, n)))
        B = f32(rng.standard_normal((n, p)))
        decs.append(c.decompose(gpu(A), "circulant", K))
        Bs.append(gpu(B))
        if m == n:
            wants.append(np.real(oc.apply_zeroth(oc.CirculantDecomp(A, K), B)))
        else:
            wants.append(oc.apply_blocked(oc.BlockedCirculant(A, K), B))
    plan = c.batch_plan(decs, Bs)
    eager = [o.clone() for o in plan.run(use_graph=False)]
    torch.cuda.synchronize()
    for o, w in zip(eager, wants):
        assert rel(host(o), w) < TOL_F32
    for rep in range(3):
        for o in plan.outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.run(use_graph=True)
        torch.cuda.synchronize()
        for o, e in zip(plan.outs, eager):
            assert torch.equal(o, e), f"replay {rep} differs"
    n = 2049
    d = c.decompose(gpu(_toeplitz(n, 3)), "circulant", 3)
    with pytest.raises(AmmError):
        c.batch_plan([d], [gpu(np.ones((n, 4)))])

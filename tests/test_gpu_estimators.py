"""Error estimates of the first-order product (Sec. 2.5, Sec. 3) through the C
ABI against the float64 oracle: the circulant concentration mu, the sketch's
sigma_{k+1}, the prior / posterior / Thm. 3.8 / circulant estimates, the
randomized sketch, and the rank choice."""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import estimators as oe
from oracle import product as op
from oracle import tsvd as ot
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu


def _toeplitz(n, seed, noise=0.05):
    rng = np.random.default_rng(seed)
    return f32(inputs.toeplitz_uniform(n, rng) + noise * rng.standard_normal((n, n)))


def _close(a, b, rtol):
    return abs(a - b) <= rtol * abs(b)


@pytest.mark.parametrize("n,K", [(64, 5), (512, 9), (2048, 33)])
def test_cd_mu_parity(n, K):
    note(f"cd mu n={n} K={K}")
    A = _toeplitz(n, n + K)
    dec = oc.CirculantDecomp(A, K)
    d = ctx().decompose(gpu(A), "circulant", K)
    assert list(d.frequencies()) == list(dec.S)
    assert _close(d.info()["mu"], oe.cd_mu(dec), 1e-9)


def test_tsvd_sigma_next_estimate():
    """The sketch's (k+1)-th singular value against the exact one.  Singular
    values of Q^T A are lower bounds (interlacing); with 16 oversampling columns
    and two subspace iterations they sit within 0.2 % here (a float64 emulation
    of the same sketch), so the test allows 0.5 % below and rounding above."""
    n, k = 512, 32
    sig = inputs.decay_power(n, 1.5)
    A = f32(inputs.spectral_matrix(n, n, sig, np.random.default_rng(4)))
    d = ctx().decompose(gpu(A), "tsvd", k, seed=3)
    s_true = np.linalg.svd(A, compute_uv=False)[k]
    got = d.info()["sigma_next"]
    assert (1 - 5e-3) * s_true <= got <= (1 + 1e-6) * s_true


def _tsvd_pair(n, k, seed):
    A = f32(inputs.spectral_matrix(n, n, inputs.decay_power(n, 1.2), np.random.default_rng(seed)))
    B = f32(inputs.spectral_matrix(n, n, inputs.decay_power(n, 1.0), np.random.default_rng(seed + 1)))
    return A, B, ot.TSVDDecomp(A, k), ot.TSVDDecomp(B, k)


def test_estimates_tsvd_imported():
    n, k = 256, 12
    A, B, decA, decB = _tsvd_pair(n, k, 30)
    c = ctx()
    Ag, Bg = gpu(A), gpu(B)
    dA = c.import_tsvd(decA.U, decA.s, decA.V, A=Ag)
    dB = c.import_tsvd(decB.U, decB.s, decB.V, A=Bg)
    sA, sB = np.linalg.svd(A, compute_uv=False), np.linalg.svd(B, compute_uv=False)
    dA.set_sigma_next(sA[k])
    dB.set_sigma_next(sB[k])
    M = c.approx_matmul(dA, Bg, dB)
    est = c.estimate_error(dA, dB, M)
    Mo = op.algorithm(decA, B, decB)
    nA, nB = np.linalg.norm(A), np.linalg.norm(B)
    ndA, ndB = decA.norm_residual(), decB.norm_residual()
    assert _close(est["norm_A"], nA, 1e-12) and _close(est["norm_B"], nB, 1e-12)
    # Delta A from float32 factors and A on the device: float32 cancellation relative to ||dA||
    assert _close(est["norm_dA"], ndA, 1e-4) and _close(est["norm_dB"], ndB, 1e-4)
    assert _close(est["prior"], oe.prior(nA, nB, ndA, ndB, n), 2e-4)
    assert _close(est["norm_M"], np.linalg.norm(Mo), TOL_F32)
    assert _close(est["posterior"], oe.posterior(ndA, ndB, np.linalg.norm(Mo), n), 2e-4)
    want_b = oe.svd_bound(ndA, ndB, sA[k], sB[k]) / np.linalg.norm(Mo)
    assert _close(est["svd_bound"], want_b, 2e-4)
    assert np.isnan(est["cd_estimate"])
    # exact factors: ||M|| <= ||AB||, so the Thm. 3.8 figure bounds the actual error
    actual = np.linalg.norm(A @ B - Mo) / np.linalg.norm(A @ B)
    assert actual <= want_b


def test_estimates_tsvd_decomposed_bound_holds():
    """Decomposed handles: sigma_next from the sketch; the Thm. 3.8 figure is
    still above the measured error (float64 AB) on this operand pair."""
    n, k = 1024, 32
    A, B, _, _ = _tsvd_pair(n, k, 40)
    c = ctx()
    Ag, Bg = gpu(A), gpu(B)
    dA = c.decompose(Ag, "tsvd", k, seed=1)
    dB = c.decompose(Bg, "tsvd", k, seed=2)
    M = c.approx_matmul(dA, Bg, dB)
    est = c.estimate_error(dA, dB, M)
    AB = A @ B
    actual = np.linalg.norm(AB - host(M)) / np.linalg.norm(AB)
    note(f"tsvd n={n} k={k}: actual {actual:.3e} prior {est['prior']:.3e} posterior {est['posterior']:.3e} "
         f"svd_bound {est['svd_bound']:.3e}")
    assert actual <= est["svd_bound"]
    sA = np.linalg.svd(A, compute_uv=False)
    assert _close(est["norm_dA"], np.sqrt(np.sum(sA[k:] ** 2)), 2e-3)


def test_estimates_circulant():
    n, K = 512, 6
    A, B = _toeplitz(n, 7), _toeplitz(n, 8)
    decA, decB = oc.CirculantDecomp(A, K), oc.CirculantDecomp(B, K)
    c = ctx()
    dA = c.decompose(gpu(A), "circulant", K)
    dB = c.decompose(gpu(B), "circulant", K)
    M = c.approx_matmul(dA, gpu(B), dB)
    for ent, code in (("signed", oe.ENTRIES_SIGNED), ("unsigned_uniform", oe.ENTRIES_UNSIGNED_UNIFORM)):
        est = c.estimate_error(dA, dB, M, entries=ent)
        Mo = np.real(op.algorithm(decA, B, decB))
        nM = np.linalg.norm(Mo)
        ndA, ndB = decA.norm_residual(), decB.norm_residual()
        assert _close(est["prior"], oe.prior(np.linalg.norm(A), np.linalg.norm(B), ndA, ndB, n, code), 1e-9)
        assert _close(est["posterior"], oe.posterior(ndA, ndB, nM, n), 2e-5)
        want = oe.cd_bound(oe.cd_mu(decA), oe.cd_mu(decB), ndA, ndB, n) / nM
        assert _close(est["cd_estimate"], want, 2e-5)
        assert np.isnan(est["svd_bound"])


def test_estimates_without_product_and_shape_errors():
    from paper_2504_19308_amd import AmmError
    n = 128
    A = _toeplitz(n, 3)
    c = ctx()
    d = c.decompose(gpu(A), "circulant", 4)
    est = c.estimate_error(d, d)
    assert np.isnan(est["posterior"]) and np.isnan(est["norm_M"]) and est["prior"] > 0
    with pytest.raises(AmmError):
        c.estimate_error(d, d, gpu(np.ones((n, n + 1))))
    tall = c.decompose(gpu(np.ones((2 * n, n))), "circulant", 4)   # 2n x n: inner dimensions differ
    with pytest.raises(AmmError):
        c.estimate_error(d, tall)


def _rademacher(p, l, seed):
    return np.random.default_rng(seed).choice([-1.0, 1.0], size=(p, l))


@pytest.mark.parametrize("n,l", [(300, 16), (4096, 32)])
def test_sketch_parity(n, l):
    """Same sketch G on both sides; the float32 products carry the 1e-5 bar,
    so |est_gpu - est| <= 1e-5 (||N|| + ||MG||) / ||N|| + 1e-5 est."""
    note(f"sketch n={n} l={l}")
    torch = torch_cuda()
    k = 32 if n >= 1024 else 8
    A, B, decA, decB = _tsvd_pair(n, k, 50 + n)
    c = ctx()
    Ag, Bg = gpu(A), gpu(B)
    dA = c.import_tsvd(decA.U, decA.s, decA.V, A=Ag)
    dB = c.import_tsvd(decB.U, decB.s, decB.V, A=Bg)
    M = c.approx_matmul(dA, Bg, dB)
    G = _rademacher(n, l, n + l)
    got = c.estimate_sketch(Ag, Bg, M, gpu(G))
    Mh = host(M)
    want = oe.sketch(A, B, Mh, G)
    N = A @ (B @ G)
    tol = 1e-5 * (np.linalg.norm(N) + np.linalg.norm(Mh @ G)) / np.linalg.norm(N) + 1e-5 * want
    assert abs(got - want) <= tol
    del torch


def test_choose_rank_circulant():
    n = 256
    A, B = _toeplitz(n, 11, 0.02), _toeplitz(n, 12, 0.02)
    c = ctx()
    dA = c.decompose(gpu(A), "circulant", 2)
    dB = c.decompose(gpu(B), "circulant", 2)
    EA, EB = oc.CirculantDecomp(A, 0).E, oc.CirculantDecomp(B, 0).E
    for ent, code in (("signed", oe.ENTRIES_SIGNED), ("unsigned_uniform", oe.ENTRIES_UNSIGNED_UNIFORM)):
        for tau in (3e-2, 1e-2, 3e-3, 1e-3):
            K = oe.choose_K_circulant(EA, EB, tau, code)
            # skip thresholds the float64 rounding of two transforms could move
            nA, nB = np.sqrt(EA.sum()), np.sqrt(EB.sum())
            def pr(k):
                return oe.prior(nA, nB, np.sqrt(max(EA.sum() - oe.retained_circulant(EA, k), 0)),
                                np.sqrt(max(EB.sum() - oe.retained_circulant(EB, k), 0)), n, code)
            if abs(pr(K) - tau) < 1e-9 * tau or (K > 0 and abs(pr(K - 1) - tau) < 1e-9 * tau):
                continue
            assert c.choose_rank(dA, dB, tau, ent) == K


def test_choose_rank_tsvd_and_adaptive_product():
    n, k = 256, 40
    A, B, decA, decB = _tsvd_pair(n, k, 60)
    c = ctx()
    Ag, Bg = gpu(A), gpu(B)
    dA = c.import_tsvd(decA.U, decA.s, decA.V, A=Ag)
    dB = c.import_tsvd(decB.U, decB.s, decB.V, A=Bg)
    nA, nB = np.linalg.norm(A), np.linalg.norm(B)
    for tau in (1e-1, 3e-2, 1e-2, 1e-3):
        want = oe.choose_k_svd(decA.s, decB.s, nA, nB, n, tau)
        assert c.choose_rank(dA, dB, tau) == want
    # adaptive: the rank chosen for 1e-2, then the first-order product at that rank
    kk = c.choose_rank(dA, dB, 1e-2)
    dA2 = c.decompose(Ag, "tsvd", kk, seed=5)
    dB2 = c.decompose(Bg, "tsvd", kk, seed=6)
    M = host(c.approx_matmul(dA2, Bg, dB2))
    err = np.linalg.norm(A @ B - M) / np.linalg.norm(A @ B)
    note(f"adaptive tsvd: k={kk} error {err:.3e}")
    assert err < 2e-2   # the prior is an estimate in expectation (Thm. 3.6), not a bound

"""Pins of the error-estimator oracle (Sec. 2.5 and Sec. 3).

Independent anchors: the deterministic bound of Thm. 3.8 as an inequality
and its flat-spectrum closed form (Cor. 3.9), the Parseval identity
sum_i X_i = ||Delta A||_F^2 for the circulant mode energies, the flat case
mu = 1 built from unit-modulus eigenvalue lists, the remark's upper bound on
mu, the claim ||M|| <= ||AB|| in the proof of Cor. 3.7, the exactness of the
sketch with G = I and the unbiasedness of its Rademacher form, Monte-Carlo
expectations for Haar (Lemma 3.1) and U(0, 1) operands (the finite-n formula
in the proof of Thm. 3.5), and an exhaustive search over K for the rank
choice.  The circulant residual theorem is checked to fail on some inputs:
it is used as an estimate, not as a bound.
"""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import estimators as oe
from oracle import tsvd as ot
from paper_2504_19308_amd import inputs


def _dense_from_lists(n, lists):
    """A = sum_k R_k D^k with r_k = F^-1 L_k, entrywise (Thm. 1.1)."""
    p = np.arange(n)[:, None]
    q = np.arange(n)[None, :]
    A = np.zeros((n, n), dtype=np.complex128)
    for k, L in lists.items():
        r = np.fft.ifft(L)
        A += r[(p - q) % n] * np.exp(2j * np.pi * ((k * q) % n) / n)
    return A


@pytest.mark.parametrize("seed", range(5))
def test_svd_bound_is_a_bound(seed):
    rng = np.random.default_rng(seed)
    n, k = 40, int(rng.integers(1, 12))
    A = inputs.spectral_matrix(n, n, inputs.decay_power(n, 0.5 + seed * 0.3), rng)
    B = rng.standard_normal((n, n))
    dA_, dB_ = ot.TSVDDecomp(A, k), ot.TSVDDecomp(B, k)
    dA, dB = dA_.residual_dense(), dB_.residual_dense()
    b = oe.svd_bound(np.linalg.norm(dA), np.linalg.norm(dB), np.linalg.norm(dA, 2), np.linalg.norm(dB, 2))
    assert np.linalg.norm(dA @ dB) <= b * (1 + 1e-12)


def test_svd_bound_flat_tail_cor39():
    """Identical residual singular values: stable rank n - k, the bound is
    ||dA|| ||dB|| / sqrt(n - k)."""
    n, k = 30, 6
    rng = np.random.default_rng(3)
    s = np.concatenate([np.linspace(10, 5, k), np.full(n - k, 0.7)])
    A = inputs.spectral_matrix(n, n, s, rng)
    B = inputs.spectral_matrix(n, n, s * 1.3, rng)
    dA, dB = ot.TSVDDecomp(A, k).residual_dense(), ot.TSVDDecomp(B, k).residual_dense()
    fa, fb = np.linalg.norm(dA), np.linalg.norm(dB)
    b = oe.svd_bound(fa, fb, np.linalg.norm(dA, 2), np.linalg.norm(dB, 2))
    assert np.isclose(b, fa * fb / np.sqrt(n - k), rtol=1e-10)
    assert np.linalg.norm(dA @ dB) <= b * (1 + 1e-12)


@pytest.mark.parametrize("n,K", [(16, 3), (32, 7), (64, 1)])
def test_cd_mode_energies_sum_to_residual(n, K):
    rng = np.random.default_rng(n + K)
    A = inputs.toeplitz_uniform(n, rng) + 0.3 * rng.standard_normal((n, n))
    dec = oc.CirculantDecomp(A, K)
    X = oe.cd_mode_energies(dec)
    assert np.isclose(np.sum(X), np.linalg.norm(np.real(dec.residual_dense())) ** 2, rtol=1e-10)
    assert oe.cd_mu(dec) >= 1.0 - 1e-12   # the maximum is at least the mean


def test_cd_mu_flat_is_one():
    """Every dropped component with unit-modulus eigenvalues: X_i is the
    number of dropped components for every mode i, so mu = 1."""
    n = 32
    rng = np.random.default_rng(9)
    neg = (-np.arange(n)) % n

    def self_conjugate():
        th = 2 * np.pi * rng.random(n)
        th[n // 2 + 1:] = -th[1:n // 2][::-1]
        th[0], th[n // 2] = 0.0, np.pi
        return np.exp(1j * th)

    lists = {0: self_conjugate(), n // 2: self_conjugate()}
    for k in range(1, n // 2):
        ph = np.exp(2j * np.pi * rng.random(n))
        lists[k] = ph
        lists[n - k] = np.conj(ph[neg])
    A = _dense_from_lists(n, lists)
    assert np.max(np.abs(A.imag)) < 1e-12
    S = [3, n - 3, 10, n - 10]
    dec = oc.CirculantDecomp(A.real, len(S), S=S)
    assert np.allclose(np.abs(np.fft.fft(dec.r, axis=0)), 1.0, atol=1e-12)
    assert np.isclose(oe.cd_mu(dec), 1.0, rtol=1e-12)
    X = oe.cd_mode_energies(dec)
    assert np.allclose(X, n - len(S), rtol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_cd_mu_below_remark_bound(seed):
    rng = np.random.default_rng(seed)
    n = 24
    A = [rng.standard_normal((n, n)), inputs.toeplitz_uniform(n, rng), np.abs(rng.standard_normal((n, n))),
         inputs.planted_circulant(n, [1, 5], rng, noise=0.1)][seed]
    dec = oc.CirculantDecomp(A, 3)
    assert oe.cd_mu(dec) <= oe.cd_mu_upper(dec) * (1 + 1e-10)


def test_cd_theorem_is_an_estimate_not_a_bound():
    """Reading: the circulant residual theorem's inequality fails on some real
    inputs (its proof drops the index shift of the conjugated components), so
    the library reports it as an estimate."""
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(200):
        n, K = 16, int(rng.integers(0, 6))
        A, B = rng.standard_normal((n, n)), rng.standard_normal((n, n))
        dA_, dB_ = oc.CirculantDecomp(A, K), oc.CirculantDecomp(B, K)
        dA, dB = np.real(dA_.residual_dense()), np.real(dB_.residual_dense())
        b = oe.cd_bound(oe.cd_mu(dA_), oe.cd_mu(dB_), np.linalg.norm(dA), np.linalg.norm(dB), n)
        worst = max(worst, np.linalg.norm(dA @ dB) / b)
    assert worst > 1.0


@pytest.mark.parametrize("k", [1, 4, 11])
def test_tsvd_first_order_norm_below_exact(k):
    """Proof of Cor. 3.7: ||M||_F <= ||AB||_F for the truncated-SVD first order."""
    rng = np.random.default_rng(k)
    n = 36
    A, B = rng.standard_normal((n, n)), inputs.spectral_matrix(n, n, inputs.decay_power(n, 1.0), rng)
    M, _, _ = ot.approx_product(A, B, k, first_order=True)
    assert np.linalg.norm(M) <= np.linalg.norm(A @ B) * (1 + 1e-12)


def test_sketch_with_identity_is_exact():
    rng = np.random.default_rng(4)
    n = 30
    A, B = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    M, _, _ = ot.approx_product(A, B, 5, first_order=True)
    exact = np.linalg.norm(A @ B - M) / np.linalg.norm(A @ B)
    assert np.isclose(oe.sketch(A, B, M, np.eye(n)), exact, rtol=1e-12)


def test_sketch_rademacher_unbiased_in_square():
    """E ||X G||_F^2 = l ||X||_F^2 for Rademacher G (n x l)."""
    rng = np.random.default_rng(8)
    n, l = 40, 8
    X = rng.standard_normal((n, n)) * np.linspace(0.1, 2, n)
    vals = [np.linalg.norm(X @ rng.choice([-1.0, 1.0], size=(n, l))) ** 2 / l for _ in range(3000)]
    assert abs(np.mean(vals) / np.linalg.norm(X) ** 2 - 1) < 0.02


def test_prior_matches_haar_monte_carlo():
    """Thm. 3.6 case 1 (Haar singular vectors): the prior estimate equals the
    ratio of expected squared norms (Lemma 3.1 in both)."""
    n, k = 96, 8
    rng = np.random.default_rng(21)
    s1, s2 = inputs.decay_power(n, 0.8), inputs.decay_exp(n, 30.0)
    num = den = 0.0
    est = []
    for _ in range(60):
        A = inputs.spectral_matrix(n, n, s1, rng)
        B = inputs.spectral_matrix(n, n, s2, rng)
        dA = ot.TSVDDecomp(A, k).residual_dense()
        dB = ot.TSVDDecomp(B, k).residual_dense()
        num += np.linalg.norm(dA @ dB) ** 2
        den += np.linalg.norm(A @ B) ** 2
        est.append(oe.prior(np.linalg.norm(A), np.linalg.norm(B), np.linalg.norm(dA), np.linalg.norm(dB), n))
    assert abs(np.sqrt(num / den) / np.mean(est) - 1) < 0.08


def test_unsigned_uniform_constant_and_prior():
    """Proof of Thm. 3.5: E||AB||^2 / (E||A||^2 E||B||^2) = 1/n + 9(n-1)/(16n)
    for U(0, 1) entries; with Haar-type residues the case-2 prior matches the
    sampled ratio ||dA dB|| / ||AB||."""
    n = 120
    rng = np.random.default_rng(5)
    r_ab, r_est = [], []
    for _ in range(40):
        A, B = rng.random((n, n)), rng.random((n, n))
        r_ab.append(np.linalg.norm(A @ B) ** 2)
        dA, dB = 0.05 * rng.standard_normal((n, n)), 0.02 * rng.standard_normal((n, n))
        got = np.linalg.norm(dA @ dB) / np.linalg.norm(A @ B)
        r_est.append(got / oe.prior(np.linalg.norm(A), np.linalg.norm(B), np.linalg.norm(dA), np.linalg.norm(dB), n,
                                    oe.ENTRIES_UNSIGNED_UNIFORM))
    expect = (1.0 / n + 9.0 * (n - 1) / (16.0 * n)) * (n * n / 3.0) ** 2
    assert abs(np.mean(r_ab) / expect - 1) < 0.01
    assert abs(np.mean(r_est) - 1) < 0.03


def test_choose_K_circulant_exhaustive():
    rng = np.random.default_rng(12)
    n = 32
    A = inputs.toeplitz_uniform(n, rng) + 0.05 * rng.standard_normal((n, n))
    B = inputs.toeplitz_uniform(n, rng) + 0.05 * rng.standard_normal((n, n))
    EA, EB = oc.CirculantDecomp(A, 0).E, oc.CirculantDecomp(B, 0).E
    nA, nB = np.linalg.norm(A), np.linalg.norm(B)
    priors = []
    for K in range(n + 1):
        dA = np.linalg.norm(np.real(oc.CirculantDecomp(A, K).residual_dense()))
        dB = np.linalg.norm(np.real(oc.CirculantDecomp(B, K).residual_dense()))
        priors.append(oe.prior(nA, nB, dA, dB, n))
    assert all(priors[i + 1] <= priors[i] * (1 + 1e-12) + 1e-15 for i in range(n))
    for tau in (1e-1, 3e-2, 1e-2, 3e-3, 1e-4):
        want = next(K for K in range(n + 1) if priors[K] <= tau * (1 + 1e-12))
        assert oe.choose_K_circulant(EA, EB, tau) == want


def test_choose_k_svd_exhaustive():
    rng = np.random.default_rng(13)
    n = 40
    A = inputs.spectral_matrix(n, n, inputs.decay_power(n, 1.5), rng)
    B = inputs.spectral_matrix(n, n, inputs.decay_power(n, 1.2), rng)
    sA, sB = np.linalg.svd(A, compute_uv=False), np.linalg.svd(B, compute_uv=False)
    for tau in (1e-1, 1e-2, 1e-3):
        want = None
        for k in range(n + 1):
            dA = np.linalg.norm(ot.TSVDDecomp(A, k).residual_dense()) if k else np.linalg.norm(A)
            dB = np.linalg.norm(ot.TSVDDecomp(B, k).residual_dense()) if k else np.linalg.norm(B)
            if oe.prior(np.linalg.norm(A), np.linalg.norm(B), dA, dB, n) <= tau:
                want = k
                break
        assert oe.choose_k_svd(sA, sB, np.linalg.norm(A), np.linalg.norm(B), n, tau) == want


def test_posterior_haar_monte_carlo_large_error():
    """Cor. 3.7 on Haar operands with flat spectra, truncated half way, where
    M and AB differ by about 13 %.  Two facts fix the expected posterior
    without using its formula: the expansion of ||M||^2 in the corollary's
    proof gives ||AB||^2 = ||M||^2 + ||dA dB||^2 for the truncated SVD, and
    Lemma 3.1 gives ||dA dB||^2 ~ ||dA||^2 ||dB||^2 / n for independent Haar
    singular vectors.  Hence posterior = ||dA|| ||dB|| / (sqrt(n) ||M||)
    ~ err / sqrt(1 - err^2), err the observed relative error; a posterior
    divided by ||AB|| would give err itself (0.50 against 0.58 here), one
    without the 1/sqrt(n) a value sqrt(n) = 8 times larger."""
    n, k = 64, 32
    rng = np.random.default_rng(31)
    post, target, err = [], [], []
    for _ in range(40):
        A = inputs.spectral_matrix(n, n, np.ones(n), rng)
        B = inputs.spectral_matrix(n, n, 2.0 * np.ones(n), rng)
        M, dA_, dB_ = ot.approx_product(A, B, k, first_order=True)
        AB = A @ B
        dA, dB = dA_.residual_dense(), dB_.residual_dense()
        nab, nm, ndd = np.linalg.norm(AB), np.linalg.norm(M), np.linalg.norm(dA @ dB)
        assert abs(nab ** 2 - nm ** 2 - ndd ** 2) <= 1e-10 * nab ** 2
        e = np.linalg.norm(AB - M) / nab
        err.append(e)
        target.append(e / np.sqrt(1.0 - e * e))
        post.append(oe.posterior(np.linalg.norm(dA), np.linalg.norm(dB), nm, n))
    assert 0.45 < np.mean(err) < 0.55
    assert abs(np.mean(post) / np.mean(target) - 1) < 0.01
    # the bound direction of Cor. 3.7 for exact truncated-SVD factors
    assert np.mean(err) <= np.mean(post)


def test_posterior_small_error_tracks_actual():
    """Fast decay, rank 8 of 96: M ~ AB and the posterior tracks the observed
    relative error of each draw (Lemma 3.1 concentrates for Haar factors)."""
    n, k = 96, 8
    rng = np.random.default_rng(32)
    ratios = []
    for _ in range(30):
        A = inputs.spectral_matrix(n, n, inputs.decay_power(n, 0.9), rng)
        B = inputs.spectral_matrix(n, n, inputs.decay_exp(n, 25.0), rng)
        M, dA_, dB_ = ot.approx_product(A, B, k, first_order=True)
        e = np.linalg.norm(A @ B - M) / np.linalg.norm(A @ B)
        p = oe.posterior(np.linalg.norm(dA_.residual_dense()), np.linalg.norm(dB_.residual_dense()),
                         np.linalg.norm(M), n)
        ratios.append(e / p)
    assert abs(np.mean(ratios) - 1) < 0.05
    assert np.std(ratios) < 0.2


def _real_flat_lists(n, support, level, rng):
    """Eigenvalues of a real circulant: modulus sqrt(level) on a support closed
    under i -> n - i, zero elsewhere, conjugate-symmetric phases."""
    lam = np.zeros(n, dtype=np.complex128)
    for i in support:
        if i == 0 or 2 * i == n:
            lam[i] = np.sqrt(level) * rng.choice([-1.0, 1.0])
        elif i < n - i:
            ph = np.exp(2j * np.pi * rng.random())
            lam[i] = np.sqrt(level) * ph
            lam[n - i] = np.conj(lam[i])
    return lam


@pytest.mark.parametrize("n,support", [(16, [0, 1, 15, 4, 12]), (32, [2, 30, 5, 27, 16]), (24, list(range(24)))])
def test_cd_bound_equality_case(n, support):
    """The circulant residual theorem is an equality when each residual is a
    single real component, Delta A = R (frequency 0) and Delta B = R' D^(n/2),
    whose eigenvalues have one common modulus on one support T (closed under
    i -> n - i) and vanish off it: then the convolution step holds with
    equality (one term per mode), the mode energies are flat on T so the
    Cauchy-Schwarz and max steps are tight, and mu = n / |T|, which is 1 only
    for a full support.  The dense product gives ||dA dB||_F independently.
    Kept components (a strong pair at frequency 3) do not change this."""
    rng = np.random.default_rng(n + len(support))
    ca, cb = 2.0, 0.5
    big = np.fft.fft(rng.standard_normal(n)) * 20.0
    neg = (-np.arange(n)) % n
    A = _dense_from_lists(n, {0: _real_flat_lists(n, support, ca, rng), 3: big, n - 3: np.conj(big[neg])})
    B = _dense_from_lists(n, {n // 2: _real_flat_lists(n, support, cb, rng)})
    assert np.max(np.abs(A.imag)) < 1e-10 and np.max(np.abs(B.imag)) < 1e-10
    decA, decB = oc.CirculantDecomp(A.real, 2), oc.CirculantDecomp(B.real, 0)
    assert sorted(decA.S.tolist()) == [3, n - 3]
    dA, dB = np.real(decA.residual_dense()), np.real(decB.residual_dense())
    muA, muB = oe.cd_mu(decA), oe.cd_mu(decB)
    assert np.isclose(muA, n / len(support), rtol=1e-10) and np.isclose(muB, n / len(support), rtol=1e-10)
    b = oe.cd_bound(muA, muB, np.linalg.norm(dA), np.linalg.norm(dB), n)
    assert np.isclose(np.linalg.norm(dA @ dB), b, rtol=1e-10)
    # closed form: ||dA dB||^2 = |T| ca cb
    assert np.isclose(b, np.sqrt(len(support) * ca * cb), rtol=1e-10)

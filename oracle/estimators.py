"""Relative-error estimators and rank choice for the first-order product, float64 (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

The quantity estimated is the relative error of the first-order product,
||AB - M||_F / ||AB||_F = ||Delta A Delta B||_F / ||AB||_F (eq. (2.1)), from
the norms the decompositions carry (Sec. 2.5 and Sec. 3):

* ``prior``       -- before any product, from ||A||, ||B||, ||Delta A||,
  ||Delta B|| (Thm. 3.6, dropping its vanishing second term): the ratio
  ||dA|| ||dB|| / (||A|| ||B||) for mean-zero entries (Haar singular
  vectors, Lemma 3.1 in numerator and denominator), and 4 / (3 sqrt(n)) times
  that ratio when A and B have unsigned U(0, a) entries (Thm. 3.5's 9/16 in
  the denominator).
* ``posterior``   -- after the product, ||dA|| ||dB|| / (sqrt(n) ||M||)
  (Cor. 3.7; an upper bound in expectation for the truncated SVD, where
  ||M|| <= ||AB||, an estimate for the other decompositions).
* ``svd_bound``   -- Thm. 3.8: ||dA dB||_F <= sqrt(||dA||_2 ||dB||_2 ||dA||_F
  ||dB||_F), with ||dA||_2 = sigma_{k+1}(A) for the best rank-k truncation.
* ``cd_mu``, ``cd_bound`` -- the circulant residual theorem of Sec. 3:
  X_i = sum_{j not kept} |lambda_i(R_j)|^2 per Fourier mode i, mu = max_i X_i /
  (||dA||_F^2 / n), and ||dA dB||_F <= (mu_A mu_B)^(1/4) ||dA|| ||dB|| / sqrt(n).
  ``cd_mu_upper`` is the remark's bound mu <= n ||cycle matrix of dA||_2^2 /
  ||dA||_F^2.
* ``sketch``      -- the randomized norm estimate of Sec. 2.5 (last item):
  ||A (B G) - M G||_F / ||A (B G)||_F with a thin n x l sketch G (N(0,1) or
  Rademacher entries, passed in).
* ``choose_K_circulant``, ``choose_k_svd`` -- the smallest truncation whose
  prior estimate meets a tolerance (Sec. 2.5: add components while the a priori
  estimate is not small enough); one K for both operands, as Alg. 2.3 uses a
  single k.

Pins (tests/test_oracle_estimators.py): Thm. 3.8 holds as an inequality on
random and structured instances; the flat cases reduce to their closed forms
(identical residual singular values: Cor. 3.9; flat Fourier energy: mu = 1);
the circulant theorem is an equality for single-component residues with
eigenvalues of one modulus on a support T (mu = n / |T|), and fails on some
other inputs (an estimate, not a bound); sum_i X_i = ||dA||_F^2 and
mu <= mu_upper; ||M|| <= ||AB|| for the truncated SVD (proof of Cor. 3.7);
the posterior matches err / sqrt(1 - err^2) on Haar operands truncated half
way (Lemma 3.1 with ||AB||^2 = ||M||^2 + ||dA dB||^2) and tracks the observed
error where it is small; the sketch with G = I is the exact ratio and its
Rademacher form is unbiased in ||.||^2; the prior estimate matches
Monte-Carlo relative errors for Haar operands and the U(0,1) constant
matches the finite-n expectation of Thm. 3.5's proof; the rank choices agree
with a search over every K.
"""
from __future__ import annotations

import numpy as np

from . import circulant as oc

ENTRIES_SIGNED = 0             # mean-zero entries / Haar singular vectors
ENTRIES_UNSIGNED_UNIFORM = 1   # U(0, a) entries


def prior(norm_A: float, norm_B: float, norm_dA: float, norm_dB: float, n: int,
          entries: int = ENTRIES_SIGNED) -> float:
    """Thm. 3.6 without its O(1/sqrt(n)) term (epsilon -> 0)."""
    if norm_A == 0.0 or norm_B == 0.0:
        return 0.0 if norm_dA * norm_dB == 0.0 else float("inf")
    ratio = norm_dA * norm_dB / (norm_A * norm_B)
    if entries == ENTRIES_SIGNED:
        return float(ratio)
    if entries == ENTRIES_UNSIGNED_UNIFORM:
        return float(4.0 / (3.0 * np.sqrt(n)) * ratio)
    raise ValueError("entries")


def posterior(norm_dA: float, norm_dB: float, norm_M: float, n: int) -> float:
    """Cor. 3.7: ||dA|| ||dB|| / (sqrt(n) ||M||), M the first-order product."""
    if norm_M == 0.0:
        return 0.0 if norm_dA * norm_dB == 0.0 else float("inf")
    return float(norm_dA * norm_dB / (np.sqrt(n) * norm_M))


def svd_bound(norm_dA: float, norm_dB: float, spec_dA: float, spec_dB: float) -> float:
    """Thm. 3.8: upper bound on ||dA dB||_F (absolute)."""
    return float(np.sqrt(spec_dA * spec_dB * norm_dA * norm_dB))


def cd_mode_energies(dec: oc.CirculantDecomp) -> np.ndarray:
    """X_i = sum over dropped j of |lambda_i(R_j)|^2 (definition before the
    circulant theorem); lambda_i(R_j) are the entries of F r_{., j}."""
    n = dec.n
    lam = np.fft.fft(dec.r, axis=0)          # column j: eigenvalues of R_j
    keep = np.zeros(n, dtype=bool)
    keep[dec.S] = True
    return np.sum(np.abs(lam[:, ~keep]) ** 2, axis=1)


def cd_mu(dec: oc.CirculantDecomp) -> float:
    """Spectral concentration parameter mu of Delta A."""
    X = cd_mode_energies(dec)
    tot = float(np.sum(X))
    if tot == 0.0:
        return 1.0
    return float(np.max(X) / (tot / dec.n))


def cd_mu_upper(dec: oc.CirculantDecomp) -> float:
    """Remark before the circulant theorem: mu <= n ||cycle matrix of dA||_2^2 / ||dA||_F^2."""
    dA = np.real(dec.residual_dense())
    f2 = float(np.sum(dA * dA))
    if f2 == 0.0:
        return 1.0
    und = oc.cycle_matrix(dA)
    return float(dec.n * np.linalg.norm(und, 2) ** 2 / f2)


def cd_bound(mu_A: float, mu_B: float, norm_dA: float, norm_dB: float, n: int) -> float:
    """Circulant residual theorem: upper bound on ||dA dB||_F (absolute)."""
    return float((mu_A * mu_B) ** 0.25 / np.sqrt(n) * norm_dA * norm_dB)


def sketch(A: np.ndarray, B: np.ndarray, M: np.ndarray, G: np.ndarray) -> float:
    """||A(BG) - MG||_F / ||A(BG)||_F (Sec. 2.5, randomized Frobenius norms)."""
    A, B, M, G = (np.asarray(x, dtype=np.float64) for x in (A, B, M, G))
    N = A @ (B @ G)
    den = np.linalg.norm(N)
    if den == 0.0:
        return 0.0
    return float(np.linalg.norm(N - M @ G) / den)


def retained_circulant(E: np.ndarray, K: int) -> float:
    """Energy kept by the pair-closed selection of K components."""
    S = oc.select_pair_closed(E, K)
    return float(np.sum(E[S]))


def choose_K_circulant(EA: np.ndarray, EB: np.ndarray, tau: float, entries: int = ENTRIES_SIGNED) -> int:
    """Smallest K in [0, n] with prior(K) <= tau (the same K for A and B).
    ||A||^2 = sum E and ||dA(K)||^2 = sum E - retained(K) (Rem. 1.2)."""
    EA, EB = np.asarray(EA, dtype=np.float64), np.asarray(EB, dtype=np.float64)
    n = EA.size
    nA, nB = float(np.sqrt(np.sum(EA))), float(np.sqrt(np.sum(EB)))
    for K in range(n + 1):
        dA = np.sqrt(max(np.sum(EA) - retained_circulant(EA, K), 0.0))
        dB = np.sqrt(max(np.sum(EB) - retained_circulant(EB, K), 0.0))
        if prior(nA, nB, dA, dB, n, entries) <= tau:
            return K
    return n


def choose_k_svd(sA: np.ndarray, sB: np.ndarray, norm_A: float, norm_B: float, n: int, tau: float,
                 entries: int = ENTRIES_SIGNED) -> int:
    """Smallest k <= len(s) with prior(k) <= tau, ||dA(k)||^2 = ||A||^2 -
    sum_{i<k} s_i^2 (Eckart-Young); len(s) if none meets it."""
    sA, sB = np.asarray(sA, dtype=np.float64), np.asarray(sB, dtype=np.float64)
    kmax = min(sA.size, sB.size)
    for k in range(kmax + 1):
        dA = np.sqrt(max(norm_A ** 2 - np.sum(sA[:k] ** 2), 0.0))
        dB = np.sqrt(max(norm_B ** 2 - np.sum(sB[:k] ** 2), 0.0))
        if prior(norm_A, norm_B, dA, dB, n, entries) <= tau:
            return k
    return kmax

"""Pins of the Fourier-domain sparsification oracle (Sec. 2.4, Alg. 2.4/2.5).

Anchors outside the oracle: the unitary DFT built from its definition against
numpy's FFT and its unitarity, AB = F*(A) F(B); the limits k = n (exact) and
k = 0 (zero); operands whose rows are at most k/2 sinusoid pairs (kept
exactly); the first-order identity; a brute-force search over closed sets; the
literal top-k of Alg. 2.4 for even k; real products.
"""
import itertools

import numpy as np
import pytest

from oracle import sfft as osf


def _rand(m, n, seed):
    return np.random.default_rng(seed).standard_normal((m, n))


def test_dft_definition_and_parseval():
    n = 16
    W = osf.unitary_dft(n)
    assert np.allclose(W @ np.conj(W).T, np.eye(n), atol=1e-13)
    x = np.random.default_rng(1).standard_normal(n)
    assert np.allclose(W @ x, np.fft.fft(x) / np.sqrt(n), atol=1e-13)
    A, B = _rand(5, n, 2), _rand(n, 7, 3)
    d = osf.SFFTDecomp(A, n)
    assert np.allclose(d.Hrow @ (W @ B), A @ B, atol=1e-12)
    assert np.isclose(np.linalg.norm(d.Hrow), np.linalg.norm(A), rtol=1e-13)


@pytest.mark.parametrize("m,n,p", [(8, 16, 8), (12, 32, 6)])
def test_limits(m, n, p):
    A, B = _rand(m, n, m), _rand(n, p, p)
    full_A, full_B = osf.SFFTDecomp(A, n), osf.SFFTDecomp(B, n)
    assert np.allclose(osf.product(full_A, B), A @ B, atol=1e-11)
    assert np.allclose(osf.product(full_A, B, full_B), A @ B, atol=1e-11)
    zero_A, zero_B = osf.SFFTDecomp(A, 0), osf.SFFTDecomp(B, 0)
    assert np.allclose(osf.product(zero_A, B), 0.0)
    assert np.allclose(osf.product(zero_A, B, zero_B), 0.0)


def test_sparse_rows_are_kept_exactly():
    """Rows that are sums of at most k/2 real sinusoids have at most k nonzero
    frequencies, so the sparsification is exact and M0 = AB."""
    n, m, k = 64, 10, 6
    rng = np.random.default_rng(5)
    t = np.arange(n)
    A = np.zeros((m, n))
    for i in range(m):
        for f in rng.choice(np.arange(1, n // 2), size=k // 2, replace=False):
            A[i] += rng.standard_normal() * np.cos(2 * np.pi * f * t / n + rng.random() * 6)
    B = _rand(n, 9, 6)
    d = osf.SFFTDecomp(A, k)
    assert np.allclose(osf.product(d, B), A @ B, atol=1e-11)


@pytest.mark.parametrize("k", [1, 4, 7])
def test_first_order_identity_and_realness(k):
    m, n, p = 9, 32, 11
    A, B = _rand(m, n, 7 + k), _rand(n, p, 8 + k)
    dA, dB = osf.SFFTDecomp(A, k), osf.SFFTDecomp(B, k)
    M = osf.product_complex(dA, B, dB)
    assert np.max(np.abs(M.imag)) < 1e-10 * np.max(np.abs(M.real))
    FA_res = dA.Hrow - dA.left_sparse()
    FB_res = dB.Hcol - dB.right_sparse()
    assert np.allclose(M.real, A @ B - np.real(FA_res @ FB_res), atol=1e-11)


def test_selection_bruteforce_small():
    """Among all closed sets of at most k frequencies, the kept set retains
    the most energy in each row."""
    n = 8
    A = _rand(6, n, 11)
    classes = [[0], [n // 2]] + [[q, n - q] for q in range(1, n // 2)]
    for k in range(n + 1):
        d = osf.SFFTDecomp(A, k)
        for i in range(A.shape[0]):
            E = np.abs(d.Hrow[i]) ** 2
            best = 0.0
            for r in range(len(classes) + 1):
                for combo in itertools.combinations(classes, r):
                    idx = [q for c in combo for q in c]
                    if len(idx) <= k:
                        best = max(best, E[idx].sum())
            assert np.isclose(E[d.row_mask[i]].sum(), best, rtol=1e-12)
            assert d.row_mask[i].sum() <= k


def test_even_k_matches_literal_topk():
    """Alg. 2.4 as printed agrees with the closed selection for even k when
    the magnitudes are exactly symmetric, untied at the cut, and neither
    self-conjugate frequency (0, n/2) is among the k largest."""
    m, n = 40, 32
    A = _rand(m, n, 12)
    H = np.fft.ifft(A, axis=1) * np.sqrt(n)          # A W* through numpy
    Hs = 0.5 * (H + np.conj(H[:, (-np.arange(n)) % n]))   # exact conjugate symmetry
    checked = 0
    for k in (2, 6, 10):
        lit = osf.select_literal_rows(Hs, k)
        closed = osf.select_rows(Hs, k)
        for i in range(m):
            mags = np.sort(np.abs(Hs[i]))[::-1]
            if np.isclose(mags[k - 1], mags[k], rtol=1e-9) or lit[i, 0] or lit[i, n // 2]:
                continue
            assert np.array_equal(lit[i], closed[i])
            checked += 1
    assert checked > 50


def test_sampled_entries_match_dense_product():
    m, n, p, k = 12, 32, 10, 5
    A, B = _rand(m, n, 21), _rand(n, p, 22)
    rows, cols = np.array([0, 3, 11]), np.array([1, 2, 9])
    for first in (False, True):
        full = osf.product(osf.SFFTDecomp(A, k), B, osf.SFFTDecomp(B, k) if first else None)
        part = osf.product_entries(A, B, k, rows, cols, first)
        assert np.allclose(part, full[np.ix_(rows, cols)], atol=1e-12)

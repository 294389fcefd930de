"""Fourier-domain sparsification and its first-order product, float64 (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

Sec. 2.4 (Alg. 2.4 and 2.5): with the unitary DFT W[p, q] = exp(-2 pi i p q / n)
/ sqrt(n) over the inner dimension n,
    AB = F*(A) F(B),   F*(A) = A W*,   F(B) = W B.
F*(A) is sparsified to its k dominant frequencies in each row, F(B) to its k
dominant frequencies in each column, and the first-order product is
    M = Atil F(B) + (F*(A) - Atil) Btil,
the zeroth-order product M0 = Atil F(B).

Reading (as for the circulant selection): for real A every row of F*(A) is
conjugate-symmetric, |F*(A)[i, q]| = |F*(A)[i, n - q]|, and a set that keeps q
but not n - q makes the product complex.  Each row (column) keeps the closed
set of at most k frequencies {q, n - q} with the largest retained energy --
the rule of ``circulant.select_pair_closed`` applied to |.|^2 of that row.
When k is even and no two classes tie at the cut, this is exactly the literal
top-k of Alg. 2.4 (equal magnitudes come in pairs).  Alg. 2.5 calls Alg. 2.4
"by row" on F(B) while the text says columns; columns are used (the text).

Pins (tests/test_oracle_sfft.py): Parseval (W unitary) and AB = F*(A) F(B);
k = n reproduces AB, k = 0 gives zero; rows made of at most k/2 sinusoid
pairs are kept exactly, so M0 = AB; the first-order identity
M = AB - (F*(A) - Atil)(F(B) - Btil); the selection against a brute-force
search over closed sets and against the literal top-k for even k; and the
product is real.
"""
from __future__ import annotations

import numpy as np

from . import circulant as _circ


def unitary_dft(n: int) -> np.ndarray:
    """W[p, q] = exp(-2 pi i p q / n) / sqrt(n), built from its definition."""
    p = np.arange(n)[:, None]
    q = np.arange(n)[None, :]
    return np.exp(-2j * np.pi * ((p * q) % n) / n) / np.sqrt(n)


def select_rows(H: np.ndarray, k: int) -> np.ndarray:
    """Boolean mask of the kept entries: per row, the pair-closed selection of
    at most k frequencies by |H|^2."""
    mask = np.zeros(H.shape, dtype=bool)
    k = min(k, H.shape[1])            # Alg. 2.4: k = min(k, n)
    for i in range(H.shape[0]):
        E = np.abs(H[i]) ** 2
        mask[i, _circ.select_pair_closed(E, k)] = True
    return mask


def select_literal_rows(H: np.ndarray, k: int) -> np.ndarray:
    """Alg. 2.4 as printed: the k largest |H| of each row (ties: smaller index)."""
    mask = np.zeros(H.shape, dtype=bool)
    n = H.shape[1]
    for i in range(H.shape[0]):
        order = np.lexsort((np.arange(n), -np.abs(H[i])))
        mask[i, order[:min(k, n)]] = True
    return mask


class SFFTDecomp:
    """F*(A) = A W* sparsified by rows (left operand) and F(A) = W A sparsified
    by columns (right operand) -- a handle serves either role."""

    def __init__(self, A, k: int):
        A = np.asarray(A, dtype=np.float64)
        self.A = A
        self.k = int(k)
        m, n = A.shape
        self.W_in = unitary_dft(n)           # for the left role (inner dimension n)
        self.W_out = unitary_dft(m)          # for the right role (inner dimension m)
        self.Hrow = A @ np.conj(self.W_in).T  # F*(A), rows sparsified
        self.row_mask = select_rows(self.Hrow, k)
        self.Hcol = self.W_out @ A           # F(A), columns sparsified
        self.col_mask = select_rows(self.Hcol.T, k).T

    def left_sparse(self) -> np.ndarray:
        return np.where(self.row_mask, self.Hrow, 0.0)

    def right_sparse(self) -> np.ndarray:
        return np.where(self.col_mask, self.Hcol, 0.0)


def product(decA: SFFTDecomp, B: np.ndarray, decB: SFFTDecomp | None = None) -> np.ndarray:
    """M0 = Atil F(B), or M = Atil F(B) + (F*(A) - Atil) Btil (Alg. 2.5); the
    real part (the closed selections make it real up to rounding)."""
    B = np.asarray(B, dtype=np.float64)
    FB = decA.W_in @ B
    At = decA.left_sparse()
    M = At @ FB
    if decB is not None:
        M = M + (decA.Hrow - At) @ decB.right_sparse()
    return np.real(M)


def product_complex(decA: SFFTDecomp, B: np.ndarray, decB: SFFTDecomp | None = None) -> np.ndarray:
    """The same without taking the real part (for the realness pin)."""
    B = np.asarray(B, dtype=np.float64)
    FB = decA.W_in @ B
    At = decA.left_sparse()
    M = At @ FB
    if decB is not None:
        M = M + (decA.Hrow - At) @ decB.right_sparse()
    return M


def product_entries(A: np.ndarray, B: np.ndarray, k: int, rows, cols, first_order: bool = True) -> np.ndarray:
    """M[rows][:, cols] of Alg. 2.5 from the needed rows of F*(A) and columns of
    F(B) only (numpy's FFT per vector: F*(A)[i] = sqrt(n) ifft(A[i]), F(B)[:, j]
    = fft(B[:, j]) / sqrt(n)); the same selection rule as ``select_rows``."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    n = A.shape[1]
    Ha = np.fft.ifft(A[rows], axis=1) * np.sqrt(n)
    Hb = np.fft.fft(B[:, cols], axis=0) / np.sqrt(n)
    ma = select_rows(Ha, k)
    At = np.where(ma, Ha, 0.0)
    M = At @ Hb
    if first_order:
        mb = select_rows(Hb.T, k).T
        M = M + (Ha - At) @ np.where(mb, Hb, 0.0)
    return np.real(M)

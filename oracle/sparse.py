"""Dominant-entry sparsification with a truncated dense residue (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

The paper splits each operand into a sparse part of few dominant entries plus
a dense residue, A = A_s + Delta A, and multiplies to first order,
M = A_s B + Delta A B_s  (eq. (2.4), abstract).  It gives no rule for picking
the spatial dominant entries, so we read it as: the round(f m n) entries of
largest |a|, ties going to the smaller row-major index.  The dense residue
R = A - S may itself be truncated (circulant or SVD) -- the residue is then
A - (S + trunc(R)); with no truncation this is exactly eq. (2.4).

Sparse storage is CSR with column indices ascending inside each row.  The
products are plain per-row loops.

Parity pins (tests/test_oracle_tsvd_sparse.py): S B equals the dense
(A o Omega) B, f = 1 gives the exact product, f = 0 reduces to the pure
truncation, the selected set is checked against a brute-force sort of tiny
inputs, and the first-order identity M = AB - Delta A Delta B.  Omega is the
set of stored positions (``CSR.pattern``), which keeps a selected entry whose
value is exactly zero.
"""
from __future__ import annotations

import numpy as np

from . import circulant as _circ
from . import tsvd as _tsvd


class CSR:
    def __init__(self, m, n, row_ptr, col, val):
        self.m, self.n = int(m), int(n)
        self.row_ptr = np.asarray(row_ptr, dtype=np.int64)
        self.col = np.asarray(col, dtype=np.int64)
        self.val = np.asarray(val, dtype=np.float64)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        D = np.zeros((self.m, self.n))
        for i in range(self.m):
            a, b = self.row_ptr[i], self.row_ptr[i + 1]
            D[i, self.col[a:b]] = self.val[a:b]
        return D

    def pattern(self) -> np.ndarray:
        """Boolean m x n mask of the stored positions (the kept index set
        Omega), including stored entries whose value is exactly zero."""
        P = np.zeros((self.m, self.n), dtype=bool)
        for i in range(self.m):
            a, b = self.row_ptr[i], self.row_ptr[i + 1]
            P[i, self.col[a:b]] = True
        return P


def dominant_count(m: int, n: int, frac: float) -> int:
    return int(round(frac * m * n))


def extract_dominant(A: np.ndarray, nnz: int) -> CSR:
    """Keep the nnz entries of largest |a|; ties to the smaller flat index."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    flat = A.reshape(-1)
    # lexsort sorts by the last key first: primary -|a|, secondary index
    order = np.lexsort((np.arange(flat.size), -np.abs(flat)))
    keep = np.sort(order[:nnz])
    rows, cols = keep // n, keep % n
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return CSR(m, n, row_ptr, cols, flat[keep])


def spmm(S: CSR, B: np.ndarray) -> np.ndarray:
    """S B with one loop over rows and their stored entries."""
    B = np.asarray(B, dtype=np.float64)
    out = np.zeros((S.m, B.shape[1]))
    for i in range(S.m):
        for e in range(S.row_ptr[i], S.row_ptr[i + 1]):
            out[i, :] += S.val[e] * B[S.col[e], :]
    return out


def dense_times_sparse(D: np.ndarray, S: CSR) -> np.ndarray:
    """D S, looping over the stored entries of S (row j of S feeds column c)."""
    # a complex D (a circulant residual) keeps its real part: S is real
    D = np.real(np.asarray(D)).astype(np.float64)
    out = np.zeros((D.shape[0], S.n))
    for j in range(S.m):
        for e in range(S.row_ptr[j], S.row_ptr[j + 1]):
            out[:, S.col[e]] += D[:, j] * S.val[e]
    return out


class SparseDecomp:
    """A = S + trunc(R) + Delta A, with trunc in {None, 'circulant', 'tsvd'}."""

    def __init__(self, A, frac: float, trunc: str | None = None, K: int = 0,
                 nnz: int | None = None):
        A = np.asarray(A, dtype=np.float64)
        self.A = A
        m, n = A.shape
        self.S = extract_dominant(A, dominant_count(m, n, frac) if nnz is None else nnz)
        self.R = A - self.S.dense()
        self.trunc = trunc
        if trunc is None:
            self.inner = None
        elif trunc == "circulant":
            self.inner = _circ.CirculantDecomp(self.R, K)
        elif trunc == "tsvd":
            self.inner = _tsvd.TSVDDecomp(self.R, K)
        else:
            raise ValueError(trunc)

    def truncated_dense(self) -> np.ndarray:
        T = self.S.dense()
        if self.inner is not None:
            T = T + np.real(self.inner.truncated_dense())
        return T

    def residual_dense(self) -> np.ndarray:
        return self.A - self.truncated_dense()


def apply_zeroth(dec: SparseDecomp, B) -> np.ndarray:
    """(S + trunc(R)) B: row loops for S, the truncation's own path for R."""
    out = spmm(dec.S, B)
    if dec.inner is not None:
        if dec.trunc == "circulant":
            out = out + np.real(_circ.apply_zeroth(dec.inner, B))
        else:
            out = out + _tsvd.apply_zeroth(dec.inner, B)
    return out


def apply_first_order_term(decB: SparseDecomp, dA) -> np.ndarray:
    """Delta A (S_B + trunc(R_B))."""
    out = dense_times_sparse(dA, decB.S)
    if decB.inner is not None:
        if decB.trunc == "circulant":
            out = out + np.real(_circ.apply_first_order_term(decB.inner, dA))
        else:
            out = out + _tsvd.apply_first_order_term(decB.inner, dA)
    return out

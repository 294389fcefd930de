"""Circulant decomposition and its approximate product, float64 (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

Conventions (Sec. 1.2.2-1.2.3 of the paper, Thm. 1.1):
  * C is the full-cycle permutation with C[0, n-1] = 1 and C[i, i-1] = 1, so
    C^j has its one in row r at column (r - j) mod n.
  * D = diag(w^q) with w = exp(+2 pi i / n)  (Thm. 1.1's sign).
  * W is the unitary DFT, W[p, q] = exp(-2 pi i p q / n) / sqrt(n); the
    unnormalised forward transform F = sqrt(n) W is numpy's ``fft``, and the
    inverse carries the 1/n (numpy's ``ifft``).
  * Right cycle decomposition A = sum_j C^j Lambda_j with
    Lambda_j(l, l) = A[(l + j) mod n, l]; the cycle matrix holds cycle j in
    column j: Aund[l, j] = A[(l + j) mod n, l]   (appendix, Alg. A.2).
  * r[j, k] = (1/n) sum_l w^(-k l) Lambda_j(l, l)  (proof of Thm. 1.1,
    Alg. 2.2), R_k the circulant with r[., k] on its cycles, A = sum_k R_k D^k.

Selection reading (the paper ranks by ||R_k^(0)||_2 and takes the top k,
Alg. 2.3 steps 2-3, without saying what happens to conjugate pairs): for real
A, T[k] = T[n-k], and a set that keeps k but not n-k makes the truncated
matrix complex.  We keep whole classes {k, n-k} and, among all such closed
sets of at most K members, take the one that retains the most energy -- the
closed counterpart of "top K", since the dropped energy is exactly
||Delta A||_F^2 (Rem. 1.2).  There are at most two singleton classes ({0} and
{n/2}), so the optimum is found by trying each subset of singletons and
filling the rest of the budget with the highest-energy pairs (class energy
E[k] + E[n-k], ties to the smaller k).  Ties between candidate sets go to the
larger set, then to the order {}, {0}, {n/2}, {0, n/2}.  ``select_literal``
gives the literal top-K for comparison.

Parity pins (tests/test_oracle_circulant.py): reconstruction with all n
components (Thm. 1.1), Parseval / Frobenius orthogonality (Rem. 1.2),
diagonalisation by the DFT built from its definition, the shift identity
W D^k W* = C^k, the printed n = 4 cycle-matrix example, Thm. 2.1 optimality,
special cases (circulant input, single planted mode), and a brute-force
comparison of the algorithm path against the dense entrywise truncated
product for every index set at n <= 8.  The magnitudes T[k] are checked
against components found by orthogonal projection onto span{C^j D^k}, and the
literal top-K against an exhaustive search over K-subsets.  Blocked rectangular operands: all
components of every block reproduce A and AB exactly, a square operand is a
single block, and the block-by-block product equals the cropped dense
truncated matrix times B.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Cycle decomposition (appendix, Alg. A.2)
# ---------------------------------------------------------------------------
def cycle_matrix(A: np.ndarray) -> np.ndarray:
    """Aund[l, j] = A[(l + j) mod n, l]: column j is the diagonal of Lambda_j."""
    A = np.asarray(A)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("cycle decomposition needs a square matrix")
    Aund = np.empty_like(A)
    l = np.arange(n)
    for j in range(n):
        Aund[:, j] = A[(l + j) % n, l]
    return Aund


def permutation_C(n: int) -> np.ndarray:
    """Full-cycle permutation of eq. (1.1): ones at (0, n-1) and (i, i-1)."""
    C = np.zeros((n, n))
    C[0, n - 1] = 1.0
    for i in range(1, n):
        C[i, i - 1] = 1.0
    return C


def phase_D(n: int, k: int = 1) -> np.ndarray:
    """D^k = diag(w^(k q)), w = exp(+2 pi i / n)  (Thm. 1.1)."""
    q = np.arange(n)
    return np.diag(np.exp(2j * np.pi * ((k * q) % n) / n))


def unitary_W(n: int) -> np.ndarray:
    """W[p, q] = exp(-2 pi i p q / n) / sqrt(n)  (Rem. 1.2)."""
    p = np.arange(n)
    return np.exp(-2j * np.pi * ((p[:, None] * p[None, :]) % n) / n) / np.sqrt(n)


# ---------------------------------------------------------------------------
# Circulant decomposition via FFT (Alg. 2.2)
# ---------------------------------------------------------------------------
def circulant_coefficients(A: np.ndarray) -> np.ndarray:
    """All r[j, k], shape (n, n), index [cycle j, frequency k]   (Alg. 2.2).

    Step 1 builds the cycle matrix, step 2 takes B_ = W Aund along columns,
    and R(k) = B_(k, :)^T / sqrt(n) is the first column of R_k.
    """
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    Aund = cycle_matrix(A)
    Bund = np.fft.fft(Aund, axis=0) / np.sqrt(n)      # W applied to columns
    return (Bund / np.sqrt(n)).T                     # [j, k] = Bund[k, j]/sqrt(n)


def magnitudes(r: np.ndarray) -> np.ndarray:
    """T[k] = ||R_k^(0)||_2, the 2-norm of the first column (Alg. 2.3 step 2)."""
    return np.sqrt(np.sum(np.abs(r) ** 2, axis=0))


def energies(r: np.ndarray) -> np.ndarray:
    """||R_k||_F^2 = n T[k]^2  (each of the n cycles of R_k repeats r[j,k])."""
    n = r.shape[0]
    return n * np.sum(np.abs(r) ** 2, axis=0)


def select_pair_closed(E: np.ndarray, K: int) -> np.ndarray:
    """Closed frequency set of at most K members retaining the most energy.

    See the module header for the reading.  Returns the kept frequencies in
    ascending order.
    """
    n = len(E)
    if K < 0 or K > n:
        raise ValueError("K out of range")
    singles = [0] + ([n // 2] if n % 2 == 0 and n > 1 else [])
    pairs = [k for k in range(1, (n + 1) // 2)]
    pairs.sort(key=lambda k: (-(E[k] + E[n - k]), k))
    subsets = [[]] + [[s] for s in singles]
    if len(singles) == 2:
        subsets.append(list(singles))
    best = None
    for U in subsets:
        if len(U) > K:
            continue
        P = pairs[: (K - len(U)) // 2]
        members = list(U) + [m for k in P for m in (k, n - k)]
        total = float(sum(E[m] for m in members))
        key = (total, len(members))
        if best is None or key > best[0]:
            best = (key, members)
    return np.array(sorted(best[1]), dtype=np.int64)


def select_literal(T: np.ndarray, K: int) -> np.ndarray:
    """Literal top-K of T (ties to the smaller index), Alg. 2.3 step 3."""
    order = sorted(range(len(T)), key=lambda k: (-T[k], k))
    return np.array(order[:K], dtype=np.int64)


def eigen_lists(r: np.ndarray, S) -> np.ndarray:
    """L[t] = sqrt(n) W R[S[t]] = F r[., S[t]]   (Alg. 2.3 step 4)."""
    S = np.asarray(S, dtype=np.int64)
    if len(S) == 0:
        return np.zeros((0, r.shape[0]), dtype=np.complex128)
    return np.fft.fft(r[:, S], axis=0).T


class CirculantDecomp:
    """Truncated circulant decomposition of one square operand."""

    def __init__(self, A, K: int, literal: bool = False, S=None):
        A = np.asarray(A, dtype=np.float64)
        self.A = A
        self.n = A.shape[0]
        self.r = circulant_coefficients(A)
        self.E = energies(self.r)
        if S is not None:
            self.S = np.asarray(S, dtype=np.int64)
        elif literal:
            self.S = select_literal(magnitudes(self.r), K)
        else:
            self.S = select_pair_closed(self.E, K)
        self.L = eigen_lists(self.r, self.S)

    # -- dense entrywise truncated matrix (definition of Thm. 1.1) ----------
    def truncated_dense(self) -> np.ndarray:
        """Atil[p, q] = sum_{k in S} r[(p - q) mod n, k] w^(k q)."""
        n = self.n
        p = np.arange(n)[:, None]
        q = np.arange(n)[None, :]
        At = np.zeros((n, n), dtype=np.complex128)
        for k in self.S:
            At += self.r[(p - q) % n, k] * np.exp(2j * np.pi * ((k * q) % n) / n)
        return At

    def residual_dense(self) -> np.ndarray:
        """Delta A = A - sum_{t in S} R_t D^t  (Alg. 2.3 step 6, first line)."""
        return self.A - self.truncated_dense()

    def norm_residual(self) -> float:
        """||Delta A||_F from the discarded energies (Rem. 1.2)."""
        keep = np.zeros(self.n, dtype=bool)
        keep[self.S] = True
        return float(np.sqrt(max(np.sum(self.E[~keep]), 0.0)))


# ---------------------------------------------------------------------------
# Products (Alg. 2.3 steps 5 and 6)
# ---------------------------------------------------------------------------
def apply_zeroth(dec: CirculantDecomp, B: np.ndarray) -> np.ndarray:
    """sum_t R_t D^(k_t) B = IFFT( sum_t diag(L_t) C^(k_t) FFT(B) )   (step 5)."""
    B = np.asarray(B, dtype=np.complex128)
    n = dec.n
    Xh = np.fft.fft(B, axis=0)
    Z = np.zeros_like(Xh)
    p = np.arange(n)
    for t, k in enumerate(dec.S):
        Z += dec.L[t][:, None] * Xh[(p - k) % n, :]      # (C^k X)[p] = X[p-k]
    return np.fft.ifft(Z, axis=0)


def apply_first_order_term(decB: CirculantDecomp, dA: np.ndarray) -> np.ndarray:
    """Delta A . Btil = ( IFFT( sum_t (C^k_t)^* diag(conj L_t) FFT(Delta A^*) ) )^*
    (Alg. 2.3 step 6, second line); (C^k)^* v [p] = v[(p + k) mod n]."""
    n = decB.n
    Y = np.fft.fft(np.conj(np.asarray(dA, dtype=np.complex128)).T, axis=0)
    Z = np.zeros_like(Y)
    p = np.arange(n)
    for t, k in enumerate(decB.S):
        idx = (p + k) % n
        Z += np.conj(decB.L[t][idx])[:, None] * Y[idx, :]
    return np.conj(np.fft.ifft(Z, axis=0)).T


# ---------------------------------------------------------------------------
# Rectangular operands in square blocks (Sec. 2.3: rectangular matrices are
# approximated through square blocks).  Reading: s = min(m, n); the longer
# dimension is cut into ceil(max(m, n) / s) blocks of s, the last one padded
# with zeros; each block keeps its own K components.  Zeroth order only.
# ---------------------------------------------------------------------------
class BlockedCirculant:
    """Truncated circulant decompositions of the s x s blocks of an m x n A."""

    def __init__(self, A, K: int):
        A = np.asarray(A, dtype=np.float64)
        self.m, self.n = A.shape
        self.s = min(self.m, self.n)
        self.rows = self.m > self.n            # blocks stacked down the rows
        long = max(self.m, self.n)
        self.nb = -(-long // self.s)
        self.blocks = []
        for j in range(self.nb):
            blk = np.zeros((self.s, self.s))
            lo, hi = j * self.s, min(long, (j + 1) * self.s)
            if self.rows:
                blk[: hi - lo, :] = A[lo:hi, :]
            else:
                blk[:, : hi - lo] = A[:, lo:hi]
            self.blocks.append(CirculantDecomp(blk, K))

    def truncated_dense(self) -> np.ndarray:
        """The m x n truncated matrix: the blocks' truncations, padding cut off."""
        parts = [np.real(b.truncated_dense()) for b in self.blocks]
        full = np.vstack(parts) if self.rows else np.hstack(parts)
        return full[: self.m, : self.n]


def apply_blocked(dec: BlockedCirculant, B: np.ndarray) -> np.ndarray:
    """Atil B block by block (Alg. 2.3 step 5 on each block)."""
    B = np.asarray(B, dtype=np.float64)
    s = dec.s
    if dec.rows:
        out = np.vstack([np.real(apply_zeroth(b, B)) for b in dec.blocks])
        return out[: dec.m]
    out = np.zeros((dec.m, B.shape[1]))
    for j, b in enumerate(dec.blocks):
        Bj = np.zeros((s, B.shape[1]))
        lo, hi = j * s, min(dec.n, (j + 1) * s)
        Bj[: hi - lo] = B[lo:hi]
        out += np.real(apply_zeroth(b, Bj))
    return out


def approx_product(A, B, K: int, first_order: bool, KB: int | None = None,
                   SA=None, SB=None):
    """Alg. 2.3 end to end; returns (M, decA, decB)."""
    decA = CirculantDecomp(A, K, S=SA)
    M = apply_zeroth(decA, B)
    decB = None
    if first_order:
        decB = CirculantDecomp(B, K if KB is None else KB, S=SB)
        M = M + apply_first_order_term(decB, decA.residual_dense())
    return M, decA, decB

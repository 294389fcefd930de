"""Truncated-SVD approximate product, float64 (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

Sec. 2.2 of the paper: with Atil = U_A S_A V_A^T (k largest singular triplets)
and Btil = U_B S_B V_B^T, the zeroth-order product is Atil B and the
first-order product adds Delta A Btil with Delta A = A - Atil.  The oracle
forms Delta A explicitly, exactly as written; the GPU path uses the algebraic
identity Delta A U_B = A U_B - U_A S_A (V_A^T U_B) instead, so the two sides
do not share a computation.

The reference factors come from an exact SVD (LAPACK via numpy) -- not from
the randomized Alg. 2.1, which without oversampling or power iterations does
not return the best rank-k approximation.  For the generated workloads the
exact factors are also known in closed form (the generator's own Q1, sigma,
Q2), which pins this module together with the Eckart-Young identity
||A - A_k||_F = sqrt(sum_{i>k} sigma_i^2) (Sec. 2.2, relative-error formula).

The error bound of Thm. 3.8, ||dA dB||_F^2 <= ||dA||_F ||dB||_F ||dA||_2
||dB||_2, is exposed for the invariant tests; it is pinned by its flat-tail
closed form (c_A c_B)^2 (n - k) and by its equality case (rank-one residues
sharing a singular vector).
"""
from __future__ import annotations

import numpy as np


class TSVDDecomp:
    def __init__(self, A, k: int, U=None, s=None, V=None):
        A = np.asarray(A, dtype=np.float64)
        self.A = A
        self.k = int(k)
        if U is None:
            Uf, sf, Vtf = np.linalg.svd(A, full_matrices=False)
            self.sigma_all = sf
            U, s, V = Uf[:, :k], sf[:k], Vtf[:k, :].T
        else:
            self.sigma_all = None
        self.U = np.asarray(U, dtype=np.float64)
        self.s = np.asarray(s, dtype=np.float64)
        self.V = np.asarray(V, dtype=np.float64)

    def truncated_dense(self) -> np.ndarray:
        return (self.U * self.s[None, :]) @ self.V.T

    def residual_dense(self) -> np.ndarray:
        return self.A - self.truncated_dense()

    def norm_residual(self) -> float:
        """(||A||_F^2 - sum_{i<=k} sigma_i^2)^(1/2)   (Sec. 2.2)."""
        a2 = float(np.sum(self.A * self.A))
        return float(np.sqrt(max(a2 - float(np.sum(self.s ** 2)), 0.0)))


def apply_zeroth(dec: TSVDDecomp, B: np.ndarray) -> np.ndarray:
    """sum_i sigma_i u_i v_i^T B = U (S (V^T B))."""
    return dec.U @ (dec.s[:, None] * (dec.V.T @ np.asarray(B, dtype=np.float64)))


def apply_first_order_term(decB: TSVDDecomp, dA: np.ndarray) -> np.ndarray:
    """sum_i sigma_i^B Delta A w_i y_i^T = (Delta A W) S_B Y^T.

    A circulant residual arrives complex (its imaginary part is rounding for a
    real A); the factors here are real, so the real part of the product is the
    product of the real part and only that is kept.
    """
    return ((np.real(np.asarray(dA)).astype(np.float64) @ decB.U) * decB.s[None, :]) @ decB.V.T


def approx_product(A, B, k: int, first_order: bool, kB: int | None = None):
    decA = TSVDDecomp(A, k)
    M = apply_zeroth(decA, B)
    decB = None
    if first_order:
        decB = TSVDDecomp(B, k if kB is None else kB)
        M = M + apply_first_order_term(decB, decA.residual_dense())
    return M, decA, decB


def thm38_bound_sq(dA: np.ndarray, dB: np.ndarray) -> float:
    """Right-hand side of Thm. 3.8 squared-norm form."""
    fa = np.linalg.norm(dA, "fro")
    fb = np.linalg.norm(dB, "fro")
    sa = np.linalg.norm(dA, 2)
    sb = np.linalg.norm(dB, 2)
    return float(fa * fb * sa * sb)

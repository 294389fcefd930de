"""Zeroth- and first-order combination, two independent ways (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

eq. (2.1)-(2.3): with A = Atil + Delta A and B = Btil + Delta B,
  AB = Atil B + Delta A Btil + Delta A Delta B,
  M0 = Atil B                  (one-sided, zeroth order),
  M1 = Atil B + Delta A Btil   (first order) = AB - Delta A Delta B.

``algorithm`` follows each decomposition's own product steps (FFT/shift MAC,
factor products, row loops).  ``definition`` builds Atil, Btil entrywise and
multiplies dense matrices.  Tests demand the two agree to ~1e-12.

The backward of Y = P(W) X with the decomposition structure frozen (index set
S, subspaces U_k/V_k, pattern Omega held constant) is also given here: then
P is a linear projection and dX = P(W)^T dY, dW = P(dY X^T).
"""
from __future__ import annotations

import numpy as np

from . import circulant as _circ
from . import tsvd as _tsvd
from . import sparse as _sp


def _zeroth(dec, B):
    if isinstance(dec, _circ.CirculantDecomp):
        return _circ.apply_zeroth(dec, B)
    if isinstance(dec, _tsvd.TSVDDecomp):
        return _tsvd.apply_zeroth(dec, B)
    return _sp.apply_zeroth(dec, B)


def _first_term(decB, dA):
    if isinstance(decB, _circ.CirculantDecomp):
        return _circ.apply_first_order_term(decB, dA)
    if isinstance(decB, _tsvd.TSVDDecomp):
        return _tsvd.apply_first_order_term(decB, dA)
    return _sp.apply_first_order_term(decB, dA)


def algorithm(decA, B, decB=None) -> np.ndarray:
    """Product by the decompositions' own steps; real part returned."""
    M = _zeroth(decA, B)
    if decB is not None:
        M = M + _first_term(decB, decA.residual_dense())
    return np.real(M)


def definition(decA, B, decB=None) -> np.ndarray:
    """Same result from the dense truncated matrices."""
    At = np.real(decA.truncated_dense())
    M = At @ np.asarray(B, dtype=np.float64)
    if decB is not None:
        Bt = np.real(decB.truncated_dense())
        M = M + (np.asarray(decA.A, dtype=np.float64) - At) @ Bt
    return M


def rel_fro(X, Y) -> float:
    """||X - Y||_F / ||Y||_F."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    d = np.linalg.norm(Y)
    return float(np.linalg.norm(X - Y) / (d if d > 0 else 1.0))


# ---------------------------------------------------------------------------
# Frozen-structure backward
# ---------------------------------------------------------------------------
def project(dec, G: np.ndarray) -> np.ndarray:
    """P(G): the same truncation structure applied to another matrix G.

    circulant: keep G's components on the frozen index set S (orthogonal
    projection, Rem. 1.2); tsvd: U U^T G V V^T; sparse: G o Omega (+ the
    residue's own projection of G restricted off Omega).
    """
    G = np.asarray(G, dtype=np.float64)
    if isinstance(dec, _circ.CirculantDecomp):
        d = _circ.CirculantDecomp(G, 0, S=dec.S)
        return np.real(d.truncated_dense())
    if isinstance(dec, _tsvd.TSVDDecomp):
        return dec.U @ (dec.U.T @ G @ dec.V) @ dec.V.T
    if isinstance(dec, _sp.SparseDecomp):
        mask = dec.S.pattern()
        out = np.where(mask, G, 0.0)
        if dec.inner is not None:
            rest = np.where(mask, 0.0, G)
            out = out + project(dec.inner, rest)
        return out
    raise TypeError(type(dec))


def project_adjoint(dec, G: np.ndarray) -> np.ndarray:
    """P^T(G).  The circulant and SVD projections are orthogonal, hence
    self-adjoint; the sparse one, W o Omega + P_in(W o Omega^c), has the
    adjoint G o Omega + P_in(G) o Omega^c."""
    G = np.asarray(G, dtype=np.float64)
    if isinstance(dec, _sp.SparseDecomp):
        mask = dec.S.pattern()
        out = np.where(mask, G, 0.0)
        if dec.inner is not None:
            out = out + np.where(mask, 0.0, project_adjoint(dec.inner, G))
        return out
    return project(dec, G)


def backward(dec, X: np.ndarray, dY: np.ndarray):
    """(dX, dW) for Y = P(W) X with the structure of ``dec`` frozen:
    dX = P(W)^T dY and dW = P^T(dY X^T)."""
    Wt = np.real(dec.truncated_dense())
    dX = Wt.T @ np.asarray(dY, dtype=np.float64)
    dW = project_adjoint(dec, np.asarray(dY, dtype=np.float64) @ np.asarray(X, dtype=np.float64).T)
    return dX, dW

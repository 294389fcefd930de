"""Pins of the SVD, sparse and combination oracles.

Independent anchors: the generator's closed-form singular values
(Eckart-Young), the deterministic bound of Thm. 3.8, the dense first-order
identity M = AB - Delta A Delta B of eq. (2.1)-(2.3), brute-force sorting for
the dominant-entry selection, Lemma 3.1's expectation for the Haar generator,
and central finite differences for the frozen-structure gradient.
"""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import product as op
from oracle import sparse as osp
from oracle import tsvd as ot
from paper_2504_19308_amd import inputs


def _spectral(n, sigma, seed):
    return inputs.spectral_matrix(n, n, sigma, np.random.default_rng(seed))


@pytest.mark.parametrize("k", [1, 8, 31])
def test_eckart_young_closed_form(k):
    """||A - A_k||_F = sqrt(sum_{i>k} sigma_i^2) with sigma known from the
    generator (Sec. 2.2 relative-error formula)."""
    n = 64
    sigma = inputs.decay_power(n, 1.5)
    A = _spectral(n, sigma, 3)
    dec = ot.TSVDDecomp(A, k)
    assert np.allclose(dec.s, sigma[:k], rtol=1e-10)
    tail = np.sqrt(np.sum(sigma[k:] ** 2))
    assert np.isclose(np.linalg.norm(dec.residual_dense()), tail, rtol=1e-9)
    assert np.isclose(dec.norm_residual(), tail, rtol=1e-6)


def test_first_order_identity_factor_form():
    """Delta A Btil = (A U_B - U_A S_A (V_A^T U_B)) S_B V_B^T: the factor
    identity the GPU uses equals the oracle's explicit-residual form."""
    n = 48
    A = _spectral(n, inputs.decay_exp(n), 5)
    B = _spectral(n, inputs.decay_exp(n), 6)
    dA_, dB_ = ot.TSVDDecomp(A, 7), ot.TSVDDecomp(B, 9)
    H = A @ dB_.U - dA_.U @ (dA_.s[:, None] * (dA_.V.T @ dB_.U))
    want = (H * dB_.s[None, :]) @ dB_.V.T
    got = ot.apply_first_order_term(dB_, dA_.residual_dense())
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("kind", ["circulant", "tsvd", "sparse-tsvd", "sparse-circ", "sparse"])
def test_algorithm_equals_definition_and_first_order_identity(kind):
    """Both product paths agree, and M1 = AB - Delta A Delta B (eq. 2.1-2.3)."""
    n = 32
    A = _spectral(n, inputs.decay_exp(n, 5.0), 11) + 0.01 * np.random.default_rng(1).standard_normal((n, n))
    B = _spectral(n, inputs.decay_exp(n, 5.0), 12)
    if kind == "circulant":
        dA_, dB_ = oc.CirculantDecomp(A, 6), oc.CirculantDecomp(B, 5)
    elif kind == "tsvd":
        dA_, dB_ = ot.TSVDDecomp(A, 6), ot.TSVDDecomp(B, 4)
    elif kind == "sparse-tsvd":
        dA_, dB_ = osp.SparseDecomp(A, 0.05, "tsvd", 4), osp.SparseDecomp(B, 0.05, "tsvd", 3)
    elif kind == "sparse-circ":
        dA_, dB_ = osp.SparseDecomp(A, 0.05, "circulant", 4), osp.SparseDecomp(B, 0.05, "circulant", 5)
    else:
        dA_, dB_ = osp.SparseDecomp(A, 0.1), osp.SparseDecomp(B, 0.1)
    M0a = op.algorithm(dA_, B)
    M0d = op.definition(dA_, B)
    assert op.rel_fro(M0a, M0d) < 1e-12
    M1a = op.algorithm(dA_, B, dB_)
    M1d = op.definition(dA_, B, dB_)
    assert op.rel_fro(M1a, M1d) < 1e-12
    dA = A - np.real(dA_.truncated_dense())
    dB = B - np.real(dB_.truncated_dense())
    assert op.rel_fro(M1a, A @ B - dA @ dB) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_thm38_bound_holds(seed):
    """Thm. 3.8: ||dA dB||_F^2 <= ||dA||_F ||dB||_F ||dA||_2 ||dB||_2, for the
    SVD residues and (as a plain matrix inequality) the circulant ones."""
    n = 32
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    B = rng.standard_normal((n, n))
    for dA_, dB_ in ((ot.TSVDDecomp(A, 5), ot.TSVDDecomp(B, 5)),
                     (oc.CirculantDecomp(A, 5), oc.CirculantDecomp(B, 5))):
        dA = np.real(dA_.residual_dense())
        dB = np.real(dB_.residual_dense())
        lhs = np.linalg.norm(dA @ dB) ** 2
        assert lhs <= ot.thm38_bound_sq(dA, dB) * (1 + 1e-12)


def test_lemma31_haar_generator():
    """Lemma 3.1: E ||AB||_F^2 = ||D1||^2 ||D2||^2 / n for Haar factors."""
    n = 24
    rng = np.random.default_rng(77)
    s1 = inputs.decay_exp(n, 6.0)
    s2 = inputs.decay_power(n, 0.7)
    vals = []
    for _ in range(400):
        A = inputs.spectral_matrix(n, n, s1, rng)
        B = inputs.spectral_matrix(n, n, s2, rng)
        vals.append(np.linalg.norm(A @ B) ** 2)
    expect = np.sum(s1 ** 2) * np.sum(s2 ** 2) / n
    assert abs(np.mean(vals) / expect - 1) < 0.05


def test_haar_columns_orthonormal_and_sign_fixed():
    Q = inputs.haar_columns(40, 40, np.random.default_rng(5))
    assert np.max(np.abs(Q.T @ Q - np.eye(40))) < 1e-12
    M = np.random.default_rng(5).standard_normal((40, 40))
    R = Q.T @ M
    assert np.all(np.diag(R) > 0)


def test_dominant_selection_bruteforce():
    """Global top-nnz by |a|, ties to the smaller row-major index, checked
    against a plain sort of (|a| desc, index asc) on inputs with many ties."""
    rng = np.random.default_rng(4)
    A = rng.integers(-3, 4, size=(7, 9)).astype(float)
    for nnz in (0, 1, 5, 17, 40, 63):
        S = osp.extract_dominant(A, nnz)
        pairs = sorted(((-abs(A.flat[i]), i) for i in range(A.size)))
        want = sorted(i for _, i in pairs[:nnz])
        got = [r * 9 + c for r in range(7) for c in S.col[S.row_ptr[r]:S.row_ptr[r + 1]]]
        assert got == want
        assert np.array_equal(S.val, A.reshape(-1)[want])


def test_sparse_special_cases():
    n = 24
    rng = np.random.default_rng(8)
    A = rng.standard_normal((n, n))
    B = rng.standard_normal((n, n + 5))
    Bsq = rng.standard_normal((n, n))
    # S B equals (A o Omega) B
    dec = osp.SparseDecomp(A, 0.2)
    Omega = dec.S.dense() != 0
    assert np.max(np.abs(osp.spmm(dec.S, B) - np.where(Omega, A, 0) @ B)) < 1e-12
    # f = 1 keeps everything: the product is exact
    dec = osp.SparseDecomp(A, 1.0)
    assert np.max(np.abs(op.algorithm(dec, B) - A @ B)) < 1e-12
    # f = 0 reduces to the pure truncation
    decs = osp.SparseDecomp(A, 0.0, "tsvd", 5)
    dect = ot.TSVDDecomp(A, 5)
    assert op.rel_fro(op.algorithm(decs, Bsq), op.algorithm(dect, Bsq)) < 1e-12


@pytest.mark.parametrize("kind", ["circulant", "tsvd", "sparse-tsvd"])
def test_frozen_backward_finite_differences(kind):
    """dW = P^T(dY X^T), dX = P(W)^T dY for Y = P(W) X with frozen structure,
    against central differences of <P(W) X, G> along random directions."""
    n, p = 16, 10
    rng = np.random.default_rng(21)
    W = _spectral(n, inputs.decay_exp(n, 4.0), 22)
    X = rng.standard_normal((n, p))
    G = rng.standard_normal((n, p))
    if kind == "circulant":
        dec = oc.CirculantDecomp(W, 5)
    elif kind == "tsvd":
        dec = ot.TSVDDecomp(W, 4)
    else:
        dec = osp.SparseDecomp(W, 0.1, "tsvd", 3)
    dX, dW = op.backward(dec, X, G)

    def f(Wm, Xm):
        return float(np.sum(op.project(dec, Wm) @ Xm * G))

    h = 1e-6
    for _ in range(10):
        E = rng.standard_normal((n, n))
        fd = (f(W + h * E, X) - f(W - h * E, X)) / (2 * h)
        assert abs(fd - np.sum(dW * E)) <= 1e-7 * max(1.0, abs(fd))
        Ex = rng.standard_normal((n, p))
        fd = (f(W, X + h * Ex) - f(W, X - h * Ex)) / (2 * h)
        assert abs(fd - np.sum(dX * Ex)) <= 1e-7 * max(1.0, abs(fd))
    # P(W) reproduces the truncated matrix
    assert np.max(np.abs(op.project(dec, W) - np.real(dec.truncated_dense()))) < 1e-12


def _make(kind, M, K):
    if kind == "circulant":
        return oc.CirculantDecomp(M, K)
    if kind == "tsvd":
        return ot.TSVDDecomp(M, K)
    if kind == "sparse-tsvd":
        return osp.SparseDecomp(M, 0.05, "tsvd", K)
    if kind == "sparse-circ":
        return osp.SparseDecomp(M, 0.05, "circulant", K)
    return osp.SparseDecomp(M, 0.1)


@pytest.mark.parametrize("ka,kb", [("circulant", "tsvd"), ("tsvd", "circulant"), ("sparse-tsvd", "circulant"),
                                   ("circulant", "sparse-tsvd"), ("sparse", "tsvd"), ("tsvd", "sparse-circ")])
def test_mixed_decompositions_first_order_identity(ka, kb):
    """Different decompositions for A and B (admissible by eq. (2.1): the
    first-order form needs only A = Atil + Delta A and B = Btil + Delta B):
    the algorithm path equals M1 = AB - Delta A Delta B."""
    n = 32
    A = _spectral(n, inputs.decay_exp(n, 5.0), 21) + 0.01 * np.random.default_rng(2).standard_normal((n, n))
    B = _spectral(n, inputs.decay_exp(n, 5.0), 22)
    dA_, dB_ = _make(ka, A, 5), _make(kb, B, 4)
    M1 = op.algorithm(dA_, B, dB_)
    dA = A - np.real(dA_.truncated_dense())
    dB = B - np.real(dB_.truncated_dense())
    assert op.rel_fro(M1, A @ B - dA @ dB) < 1e-12
    assert op.rel_fro(M1, op.definition(dA_, B, dB_)) < 1e-12


def test_thm38_flat_tail_closed_form():
    """Flat residual spectra (Cor. 3.9's setting): the residual singular values
    are c_A and c_B (n - k of each), so ||dA||_F = c sqrt(n - k) and
    ||dA||_2 = c, and the right-hand side of Thm. 3.8 (squared form) is
    (c_A c_B)^2 (n - k), from the generator's singular values alone."""
    n, k, cA, cB = 40, 7, 0.3, 1.7
    head = np.linspace(9.0, 4.0, k)
    A = _spectral(n, np.concatenate([head, np.full(n - k, cA)]), 41)
    B = _spectral(n, np.concatenate([head * 2.0, np.full(n - k, cB)]), 42)
    dA, dB = ot.TSVDDecomp(A, k).residual_dense(), ot.TSVDDecomp(B, k).residual_dense()
    assert np.isclose(ot.thm38_bound_sq(dA, dB), (cA * cB) ** 2 * (n - k), rtol=1e-10)


def test_thm38_equality_aligned_rank_one_residues():
    """Thm. 3.8 is tight when both residues have rank one and A's dropped right
    singular vector is B's dropped left singular vector: dA = a u v^T,
    dB = b v w^T, so ||dA dB||_F^2 = (ab)^2 = ||dA||_F ||dB||_F ||dA||_2 ||dB||_2."""
    n, k, a, b = 24, 4, 0.8, 1.9
    rng = np.random.default_rng(43)
    Q1, Q2, Q3 = (inputs.haar_columns(n, n, rng) for _ in range(3))
    sA = np.zeros(n)
    sA[:k + 1] = [9.0, 7.0, 5.0, 3.0, a]
    sB = np.zeros(n)
    sB[:k + 1] = [8.0, 6.0, 4.0, 2.5, b]
    A = (Q1 * sA) @ Q2.T
    B = (Q2 * sB) @ Q3.T          # B's left singular vectors are A's right ones
    dA, dB = ot.TSVDDecomp(A, k).residual_dense(), ot.TSVDDecomp(B, k).residual_dense()
    lhs = np.linalg.norm(dA @ dB) ** 2
    assert np.isclose(lhs, (a * b) ** 2, rtol=1e-9)
    assert np.isclose(ot.thm38_bound_sq(dA, dB), lhs, rtol=1e-9)


def test_frozen_pattern_keeps_zero_valued_entries():
    """The frozen-structure reading: the frozen sparse structure is the kept index set Omega, so
    a kept entry whose value is exactly 0 stays in Omega and the projection
    P(G) = G o Omega keeps G there.  A has 5 nonzeros and 9 entries are kept,
    four of them zeros (ties at |a| = 0 go to the smallest row-major index)."""
    A = np.zeros((4, 5))
    A[0, 3], A[1, 1], A[2, 4], A[3, 0], A[3, 2] = 5.0, -4.0, 3.0, -2.0, 1.0
    dec = osp.SparseDecomp(A, 0.0, nnz=9)
    kept = sorted(r * 5 + c for r in range(4) for c in dec.S.col[dec.S.row_ptr[r]:dec.S.row_ptr[r + 1]])
    assert kept == sorted([3, 6, 14, 15, 17, 0, 1, 2, 4])
    G = np.arange(1.0, 21.0).reshape(4, 5)
    P = op.project(dec, G)
    want = np.zeros(20)
    want[kept] = G.reshape(-1)[kept]
    assert np.array_equal(P.reshape(-1), want)
    assert np.array_equal(op.project_adjoint(dec, G), P)
    # the frozen-structure gradient of <P(W) X, Y> puts dY X^T on every kept position
    rng = np.random.default_rng(44)
    X, Y = rng.standard_normal((5, 3)), rng.standard_normal((4, 3))
    _, dW = op.backward(dec, X, Y)
    assert np.count_nonzero(dW.reshape(-1)[kept]) == 9

"""Pins of the circulant oracle against what the paper and the mathematics fix.

Each test checks the oracle against something that is not the oracle's own
formula: a matrix built from the permutation C and the phase matrix D as
defined in eq. (1.1) and Thm. 1.1, the DFT matrix W from its definition,
the printed n = 4 worked example, or brute force over every index set.
"""
import itertools
import os

import numpy as np
import pytest

from oracle import circulant as oc
from paper_2504_19308_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(n, seed=0):
    return np.random.default_rng(seed).standard_normal((n, n))


def _circulant_from_C(col):
    """sum_j col[j] C^j built from powers of the permutation of eq. (1.1)."""
    n = len(col)
    C = oc.permutation_C(n)
    R = np.zeros((n, n), dtype=complex)
    P = np.eye(n)
    for j in range(n):
        R += col[j] * P
        P = C @ P
    return R


def test_worked_example_cycle_matrix_right():
    """Appendix example: printed cycle matrix of A = sum_j C^j Lambda_j."""
    gold = np.loadtxt(os.path.join(GOLD, "cycle_matrix_n4.txt"))
    i = np.arange(4)
    A = 10.0 * i[:, None] + i[None, :]
    assert np.array_equal(oc.cycle_matrix(A), gold)


def test_worked_example_left_decomposition_uses_C():
    """The printed left-decomposition example reassembles A via Lambda_j C^j,
    which pins the permutation C of eq. (1.1)."""
    gold = np.loadtxt(os.path.join(GOLD, "cycle_matrix_left_n4.txt"))
    i = np.arange(4)
    A = 10.0 * i[:, None] + i[None, :]
    C = oc.permutation_C(4)
    rebuilt = sum(np.diag(gold[:, j]) @ np.linalg.matrix_power(C, j) for j in range(4))
    assert np.array_equal(rebuilt, A)


def test_right_cycle_decomposition_reassembles():
    A = _rand(6, 1)
    Aund = oc.cycle_matrix(A)
    C = oc.permutation_C(6)
    rebuilt = sum(np.linalg.matrix_power(C, j) @ np.diag(Aund[:, j]) for j in range(6))
    assert np.allclose(rebuilt, A, atol=0, rtol=0)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 16])
def test_full_reconstruction_thm11(n):
    """Thm. 1.1: sum over all n components R_k D^k gives back A."""
    A = _rand(n, n)
    r = oc.circulant_coefficients(A)
    total = np.zeros((n, n), dtype=complex)
    for k in range(n):
        total += _circulant_from_C(r[:, k]) @ oc.phase_D(n, k)
    assert np.max(np.abs(total - A)) < 1e-13 * max(1.0, np.abs(A).max())
    dec = oc.CirculantDecomp(A, n)
    assert len(dec.S) == n
    assert np.max(np.abs(dec.truncated_dense() - A)) < 1e-13


@pytest.mark.parametrize("n", [4, 7, 16, 64])
def test_parseval_orthogonality_rem12(n):
    """Rem. 1.2: the R_k D^k are Frobenius-orthogonal, sum ||R_k||^2 = ||A||^2,
    and the residual norm equals the dropped energy."""
    A = _rand(n, 3)
    dec = oc.CirculantDecomp(A, min(5, n))
    assert np.isclose(dec.E.sum(), np.sum(A * A), rtol=1e-12)
    comps = [_circulant_from_C(dec.r[:, k]) @ oc.phase_D(n, k) for k in (0, 1, n - 1)]
    for a, b in itertools.combinations(comps, 2):
        assert abs(np.vdot(a, b)) < 1e-10 * np.sum(A * A)
    for k, c in zip((0, 1, n - 1), comps):
        assert np.isclose(np.vdot(c, c).real, dec.E[k], rtol=1e-12)
    dA = dec.residual_dense()
    assert np.isclose(np.linalg.norm(dA), dec.norm_residual(), rtol=1e-10)


@pytest.mark.parametrize("n", [4, 8, 9])
def test_dft_diagonalises_circulant(n):
    """W R_k W^* = diag(L_k)/... : with F = sqrt(n) W, F R_k F^-1 = diag(L_k)."""
    A = _rand(n, 4)
    r = oc.circulant_coefficients(A)
    W = oc.unitary_W(n)
    S = list(range(n))
    L = oc.eigen_lists(r, S)
    for k in range(n):
        Rk = _circulant_from_C(r[:, k])
        Dg = W @ Rk @ W.conj().T
        assert np.max(np.abs(Dg - np.diag(L[k]))) < 1e-12


@pytest.mark.parametrize("n", [4, 5, 8])
def test_shift_identity(n):
    """W D^k W^* = C^k (the relation used for the shift trick)."""
    W = oc.unitary_W(n)
    C = oc.permutation_C(n)
    for k in range(n):
        lhs = W @ oc.phase_D(n, k) @ W.conj().T
        assert np.max(np.abs(lhs - np.linalg.matrix_power(C, k))) < 1e-12


def test_thm21_least_squares():
    """Thm. 2.1: R_k minimises ||A - M D^k|| over circulant M; moving its
    first column by delta raises the squared error by exactly n ||delta||^2."""
    n = 8
    A = _rand(n, 5)
    r = oc.circulant_coefficients(A)
    rng = np.random.default_rng(9)
    for k in (0, 3):
        Dk = oc.phase_D(n, k)
        base = np.linalg.norm(A - _circulant_from_C(r[:, k]) @ Dk) ** 2
        delta = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        pert = np.linalg.norm(A - _circulant_from_C(r[:, k] + delta) @ Dk) ** 2
        assert np.isclose(pert - base, n * np.linalg.norm(delta) ** 2, rtol=1e-10)


def test_thm21_formula_matches():
    """R_k(j, 0) = (1/n) 1^T (A o C^j) D^-k 1  (Thm. 2.1 statement)."""
    n = 6
    A = _rand(n, 6)
    r = oc.circulant_coefficients(A)
    C = oc.permutation_C(n)
    one = np.ones(n)
    for j in range(n):
        Cj = np.linalg.matrix_power(C, j)
        for k in range(n):
            val = one @ (A * Cj) @ oc.phase_D(n, -k) @ one / n
            assert abs(val - r[j, k]) < 1e-13


def test_special_cases():
    n = 16
    rng = np.random.default_rng(2)
    # a circulant matrix has only the k = 0 component, and R_0 = A
    col = rng.standard_normal(n)
    Acirc = np.real(_circulant_from_C(col))
    dec = oc.CirculantDecomp(Acirc, 1)
    assert list(dec.S) == [0]
    assert np.sum(dec.E[1:]) < 1e-24 * np.sum(dec.E)
    assert np.max(np.abs(dec.truncated_dense() - Acirc)) < 1e-13
    # a constant matrix is circulant too
    dec = oc.CirculantDecomp(np.full((n, n), 3.0), 1)
    assert list(dec.S) == [0]
    # a planted single class {k, n-k}: two components reproduce A exactly
    A = inputs.planted_circulant(n, [3], rng)
    dec = oc.CirculantDecomp(A, 2)
    assert sorted(dec.S) == [3, n - 3]
    assert np.max(np.abs(dec.truncated_dense() - A)) < 1e-12
    # K = 0: nothing kept, zero product; first order then gives A Btil
    B = _rand(n, 7)
    dec0 = oc.CirculantDecomp(A, 0)
    assert np.max(np.abs(oc.apply_zeroth(dec0, B))) == 0.0
    decB = oc.CirculantDecomp(B, 4)
    term = oc.apply_first_order_term(decB, dec0.residual_dense())
    assert np.max(np.abs(term - A @ decB.truncated_dense())) < 1e-11


def test_real_input_symmetry():
    n = 16
    A = _rand(n, 8)
    dec = oc.CirculantDecomp(A, n)
    for k in range(1, n):
        assert np.isclose(dec.E[k], dec.E[n - k], rtol=1e-12)
    Lall = oc.eigen_lists(dec.r, list(range(n)))
    p = np.arange(n)
    for k in range(1, n):
        assert np.max(np.abs(Lall[n - k] - np.conj(Lall[k][(-p) % n]))) < 1e-12


@pytest.mark.parametrize("n", [4, 6, 8])
def test_bruteforce_all_index_sets(n):
    """Algorithm path (FFT, shifts, single inverse FFT) equals the dense
    truncated products for every index set, closed or not (complex)."""
    A = _rand(n, 10 + n)
    B = _rand(n, 20 + n)
    for size in range(n + 1):
        for S in itertools.combinations(range(n), size):
            dec = oc.CirculantDecomp(A, 0, S=list(S))
            At = dec.truncated_dense()
            M = oc.apply_zeroth(dec, B)
            assert np.max(np.abs(M - At @ B)) < 1e-12
    # first order over a sample of (SA, SB) pairs, including non-closed ones
    rng = np.random.default_rng(n)
    for _ in range(40):
        SA = sorted(rng.choice(n, size=rng.integers(0, n + 1), replace=False))
        SB = sorted(rng.choice(n, size=rng.integers(0, n + 1), replace=False))
        decA = oc.CirculantDecomp(A, 0, S=SA)
        decB = oc.CirculantDecomp(B, 0, S=SB)
        got = oc.apply_first_order_term(decB, decA.residual_dense())
        want = decA.residual_dense() @ decB.truncated_dense()
        assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("n", [5, 8, 12])
def test_selection_maximises_retained_energy(n):
    """Pair-closed selection keeps the most energy of any closed set of its
    size (exhaustive over closed sets)."""
    A = _rand(n, 30 + n)
    dec = oc.CirculantDecomp(A, n)
    E = dec.E
    classes = [[k] if (k == 0 or 2 * k == n) else [k, n - k] for k in range(n // 2 + 1)]
    for K in range(n + 1):
        S = oc.select_pair_closed(E, K)
        assert len(S) in (K, K - 1) or (K > 0 and len(S) <= K)
        assert len(set(S)) == len(S)
        for k in S:
            assert (n - k) % n in S
        got = E[S].sum()
        best = 0.0
        for mask in range(1 << len(classes)):
            members = [m for i, c in enumerate(classes) if mask >> i & 1 for m in c]
            if len(members) == len(S):
                best = max(best, E[members].sum())
        assert got >= best * (1 - 1e-12)


def test_selection_pair_closed_gives_real_product():
    n = 32
    pair = inputs.workload_toeplitz(n)
    for K in (1, 2, 3, 8):
        dec = oc.CirculantDecomp(pair.A, K)
        assert len(dec.S) in (K, K - 1)
        M = oc.apply_zeroth(dec, pair.B)
        assert np.max(np.abs(M.imag)) < 1e-10 * np.max(np.abs(M.real))


def test_toeplitz_one_component_first_order_soft():
    """Soft pin, Table 4.2 (Toeplitz & Toeplitz needs s = 1 CD-first
    component for 1% at n = 700): at n = 256 and K = 1 the first-order
    relative error is below 1%."""
    from oracle import product as op
    pair = inputs.workload_toeplitz(256)
    decA = oc.CirculantDecomp(pair.A, 1)
    decB = oc.CirculantDecomp(pair.B, 1)
    M = op.algorithm(decA, pair.B, decB)
    err = op.rel_fro(M, pair.A @ pair.B)
    assert err < 0.01


# ---- rectangular operands in square blocks ------------------------------------
@pytest.mark.parametrize("m,n", [(20, 8), (8, 21), (16, 16), (33, 4)])
def test_blocked_full_expansion_is_exact(m, n):
    """K = s keeps every component of every block: Atil = A and Atil B = AB."""
    rng = np.random.default_rng(m * 7 + n)
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((n, 5))
    dec = oc.BlockedCirculant(A, min(m, n))
    assert np.allclose(dec.truncated_dense(), A, atol=1e-12)
    assert np.allclose(oc.apply_blocked(dec, B), A @ B, atol=1e-11)


def test_blocked_square_is_one_block():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((16, 16))
    B = rng.standard_normal((16, 4))
    dec = oc.BlockedCirculant(A, 5)
    assert dec.nb == 1
    ref = oc.CirculantDecomp(A, 5)
    assert list(dec.blocks[0].S) == list(ref.S)
    assert np.allclose(oc.apply_blocked(dec, B), np.real(oc.apply_zeroth(ref, B)), atol=1e-12)


@pytest.mark.parametrize("m,n,K", [(24, 8, 3), (8, 27, 2), (40, 16, 5)])
def test_blocked_product_is_cropped_dense_truncation(m, n, K):
    """Block-by-block FFT products equal the dense truncated matrix (entrywise
    Thm. 1.1 partial sums of each padded block, padding cut off) times B."""
    rng = np.random.default_rng(m + n + K)
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((n, 6))
    dec = oc.BlockedCirculant(A, K)
    assert np.allclose(oc.apply_blocked(dec, B), dec.truncated_dense() @ B, atol=1e-11)
    # the padded rows/columns of a block never reach the product
    s = min(m, n)
    if m > n:
        last = dec.blocks[-1]
        assert last.A.shape == (s, s) and np.all(last.A[m - (dec.nb - 1) * s:] == 0)


@pytest.mark.parametrize("n", [5, 8, 12])
def test_magnitudes_by_projection(n):
    """T[k] = ||R_k e_0||_2 (Alg. 2.3 step 2) with R_k found without the
    oracle's transforms: the components R_k D^k are Frobenius-orthogonal and
    span{C^j D^k : j} has the orthogonal basis C^j D^k of norm sqrt(n)
    (Rem. 1.2), so R_k = sum_j <A, C^j D^k> / n C^j, and its first column holds
    the coefficients of C^j (C^j e_0 = e_j)."""
    A = _rand(n, 50 + n) + 0.5 * _rand(n, 60 + n) @ _rand(n, 70 + n)
    T = oc.magnitudes(oc.circulant_coefficients(A))
    C = oc.permutation_C(n)
    for k in range(n):
        Dk = oc.phase_D(n, k)
        coef = np.zeros(n, dtype=complex)
        P = np.eye(n)
        for j in range(n):
            basis = P @ Dk
            coef[j] = np.sum(np.conj(basis) * A) / n
            P = C @ P
        assert np.isclose(T[k], np.linalg.norm(coef), rtol=1e-12, atol=1e-14)


def test_select_literal_bruteforce():
    """Literal top-K (Alg. 2.3 step 3, ties to the smaller frequency): among
    all K-subsets with the largest sum of T, the lexicographically smallest;
    checked on values with many ties."""
    rng = np.random.default_rng(7)
    for n in (6, 9):
        T = rng.integers(0, 4, size=n).astype(float)
        for K in range(n + 1):
            best = max(sum(T[list(c)]) for c in itertools.combinations(range(n), K))
            want = min(c for c in itertools.combinations(range(n), K) if sum(T[list(c)]) == best)
            assert sorted(oc.select_literal(T, K).tolist()) == list(want)


def test_literal_decomposition_first_order_identity():
    """The literal selection (which may split a conjugate pair, making the
    truncation complex) still satisfies M1 = AB - Delta A Delta B entrywise."""
    n = 12
    A, B = _rand(n, 81), _rand(n, 82)
    dA_ = oc.CirculantDecomp(A, 3, literal=True)
    dB_ = oc.CirculantDecomp(B, 5, literal=True)
    assert len(dA_.S) == 3
    M1 = oc.apply_zeroth(dA_, B) + oc.apply_first_order_term(dB_, dA_.residual_dense())
    dA, dB = dA_.residual_dense(), dB_.residual_dense()
    assert np.max(np.abs(M1 - (A @ B - dA @ dB))) < 1e-10

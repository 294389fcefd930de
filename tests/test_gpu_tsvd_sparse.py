"""GPU parity of the truncated-SVD and sparse paths against the float64 oracle.

Products are compared on identical decompositions (oracle factors / CSR
imported through the C ABI) to the float32 bar 1e-5 relative Frobenius.  The
device randomized SVD is checked against what the mathematics fixes (singular
values of the generator, the Eckart-Young tail); the device extraction must
give the oracle's CSR exactly.
"""
import numpy as np
import pytest

from oracle import product as op
from oracle import sparse as osp
from oracle import tsvd as ot
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu


def _spectral(m, n, sigma, seed):
    return f32(inputs.spectral_matrix(m, n, sigma, np.random.default_rng(seed)))


@pytest.mark.parametrize("m,n,p,k", [
    (16, 16, 16, 4), (33, 47, 29, 5), (100, 64, 257, 16), (256, 256, 256, 16),
    (512, 384, 1000, 64), (1024, 1024, 1024, 128), (130, 2100, 70, 9),
])
def test_tsvd_apply_parity(m, n, p, k):
    note(f"tsvd apply m={m} n={n} p={p} k={k}")
    rng = np.random.default_rng(m + n + p)
    sig = inputs.decay_power(min(m, n), 1.0)
    A = _spectral(m, n, sig, m + 1)
    B = f32(rng.standard_normal((n, p)))
    dec = ot.TSVDDecomp(A, k)
    want = ot.apply_zeroth(dec, B)
    c = ctx()
    d = c.import_tsvd(dec.U, dec.s, dec.V)
    got = host(c.approx_matmul(d, gpu(B)))
    assert rel(got, want) < TOL_F32


@pytest.mark.parametrize("n,kA,kB,with_B", [
    (64, 4, 6, False), (256, 16, 16, False), (1024, 32, 32, False), (333, 7, 11, False),
    (256, 16, 16, True), (1024, 32, 32, True), (512, 128, 64, True), (384, 48, 16, True),
    (2048, 32, 32, True), (200, 9, 5, True)])
def test_tsvd_first_order_parity(n, kA, kB, with_B):
    """with_B: B's handle keeps Delta B, which selects the two-panel path
    M1 = U_A S_A (V_A^T Delta B) + (A U_B) S_B V_B^T when the shapes fit."""
    note(f"tsvd first order n={n} kA={kA} kB={kB} with_B={with_B}")
    sig = inputs.decay_power(n, 1.5)
    A = _spectral(n, n, sig, 11 + n)
    B = _spectral(n, n, sig, 12 + n)
    decA, decB = ot.TSVDDecomp(A, kA), ot.TSVDDecomp(B, kB)
    want = op.algorithm(decA, B, decB)
    c = ctx()
    Ag = gpu(A)
    dA = c.import_tsvd(decA.U, decA.s, decA.V, A=Ag)
    Bg = gpu(B)
    dB = c.import_tsvd(decB.U, decB.s, decB.V, A=Bg if with_B else None)
    got = host(c.approx_matmul(dA, Bg, dB))
    assert rel(got, want) < TOL_F32


@pytest.mark.parametrize("m,n,p,k", [(128, 256, 128, 16), (512, 512, 1024, 32), (2048, 2048, 2048, 128),
                                     (1024, 2048, 256, 48), (256, 4096, 512, 64)])
def test_tsvd_zeroth_fast_shapes(m, n, p, k):
    """Shapes that take the panel + short-K output GEMM path."""
    note(f"tsvd zeroth fast m={m} n={n} p={p} k={k}")
    rng = np.random.default_rng(m + 3 * k)
    sig = inputs.decay_power(min(m, n), 1.0)
    A = _spectral(m, n, sig, k)
    B = f32(rng.standard_normal((n, p)))
    dec = ot.TSVDDecomp(A, k)
    c = ctx()
    d = c.import_tsvd(dec.U, dec.s, dec.V)
    got = host(c.approx_matmul(d, gpu(B)))
    assert rel(got, ot.apply_zeroth(dec, B)) < TOL_F32


def test_tsvd_first_order_needs_A():
    from paper_2504_19308_amd import AmmError
    n = 32
    A = _spectral(n, n, inputs.decay_exp(n), 1)
    dec = ot.TSVDDecomp(A, 4)
    c = ctx()
    d = c.import_tsvd(dec.U, dec.s, dec.V)
    with pytest.raises(AmmError):
        c.approx_matmul(d, gpu(A), d)


@pytest.mark.parametrize("n,k,alpha,excess", [(256, 16, 1.5, 1e-3), (512, 32, 1.5, 1e-3),
                                              (1024, 64, 1.2, 5e-3), (600, 101, 1.5, 8e-3),
                                              (1024, 128, 1.5, 1e-2), (640, 200, 1.5, 2e-2),
                                              (160, 150, 1.5, 1e-4), (1200, 1100, 1.5, 0.12),
                                              (300, 21, 1.5, 1e-3), (40, 1, 1.5, 1e-4), (97, 81, 1.5, 1e-4)])
def test_tsvd_decompose_quality(n, k, alpha, excess):
    """Singular values of the generator are recovered and the truncation error
    is within `excess` of the Eckart-Young tail sqrt(sum_{i>k} sigma_i^2)
    (16 oversampling columns, 2 subspace iterations; the slower decay 1.2
    leaves a larger randomized-SVD excess).  Sketches above 96 columns take
    the blocked CholeskyQR and the one-sided Jacobi eigensolver: 117 columns
    (a partial 53-column block, an odd count), 144, 216, 1116 (the
    eigensolver's 4-column blocks above 1024), and 160 = min(m, n) (the
    sketch spans the whole range, so only the float32 rounding of the factors
    remains).  Odd sketch widths: 37 and 17 columns on the one-workgroup
    path (rank 21 and rank 1), 97 = min(m, n) on the blocked path (a
    33-column last Cholesky block, a 1-column last Jacobi block).  A float64
    Householder-QR randomized SVD of the same sketch size and iteration count
    leaves excesses of 3.7-4.9e-3, 5.4-6.7e-3, 0.9-1.1e-2 and 6.2-6.4e-2 on
    the four larger cases over five sketches (up to 3.5e-5 at rank 21): the
    bounds are about twice those."""
    note(f"tsvd decompose n={n} k={k}")
    sig = inputs.decay_power(n, alpha)
    A = _spectral(n, n, sig, 31 + n)
    c = ctx()
    Ag = gpu(A)
    d = c.decompose(Ag, "tsvd", k, oversample=16, power_iters=2, seed=5)
    U, s, V = d.tsvd_factors()
    s_exact = np.linalg.svd(A, compute_uv=False)
    h = max(1, k // 2)
    assert np.max(np.abs(s[:h] - s_exact[:h]) / s_exact[:h]) < 1e-5
    Ak = (U.astype(np.float64) * s.astype(np.float64)) @ V.astype(np.float64).T
    tail = np.sqrt(np.sum(s_exact[k:] ** 2))
    err = np.linalg.norm(A - Ak)
    assert err / tail - 1 < excess
    inf = d.info()
    assert np.isclose(inf["norm_A"], np.linalg.norm(A), rtol=1e-9)


@pytest.mark.parametrize("m,n,p,frac,inner,K", [
    (64, 64, 40, 0.05, None, 0), (128, 128, 128, 0.02, "tsvd", 8),
    (256, 256, 100, 0.01, "circulant", 8), (300, 200, 77, 0.03, "tsvd", 5),
])
def test_sparse_apply_parity(m, n, p, frac, inner, K):
    note(f"sparse apply m={m} n={n} frac={frac} inner={inner}")
    rng = np.random.default_rng(m * 3 + n)
    A = f32(inputs.spectral_matrix(m, n, inputs.decay_power(min(m, n), 1.5), rng))
    pos, vals = inputs.sparse_overlay(m, n, frac, 10.0, rng)
    A = A.copy()
    A.reshape(-1)[pos] += vals
    A = f32(A)
    B = f32(rng.standard_normal((n, p)))
    if inner == "circulant" and m != n:
        pytest.skip("circulant residue needs a square operand")
    dec = osp.SparseDecomp(A, frac, inner, K)
    want = osp.apply_zeroth(dec, B)
    c = ctx()
    res = None
    if inner == "tsvd":
        res = c.import_tsvd(dec.inner.U, dec.inner.s, dec.inner.V)
    elif inner == "circulant":
        res = c.import_circulant(n, dec.inner.S, dec.inner.L)
    d = c.import_sparse(m, n, dec.S.row_ptr, dec.S.col, dec.S.val, residue=res)
    got = host(c.approx_matmul(d, gpu(B)))
    assert rel(got, np.real(want)) < TOL_F32


@pytest.mark.parametrize("n,frac", [(64, 0.05), (256, 0.01)])
def test_sparse_first_order_parity(n, frac):
    rng = np.random.default_rng(n)
    mk = lambda: f32(inputs.spectral_matrix(n, n, inputs.decay_power(n, 1.5), rng))
    A, B = mk(), mk()
    for M in (A, B):
        pos, vals = inputs.sparse_overlay(n, n, frac, 10.0, rng)
        M.reshape(-1)[pos] += vals
    A, B = f32(A), f32(B)
    decA = osp.SparseDecomp(A, frac, "tsvd", 6)
    decB = osp.SparseDecomp(B, frac, "tsvd", 6)
    want = op.algorithm(decA, B, decB)
    c = ctx()
    Rg = gpu(decA.R)
    rA = c.import_tsvd(decA.inner.U, decA.inner.s, decA.inner.V, A=Rg)
    dA = c.import_sparse(n, n, decA.S.row_ptr, decA.S.col, decA.S.val, residue=rA)
    rB = c.import_tsvd(decB.inner.U, decB.inner.s, decB.inner.V)
    dB = c.import_sparse(n, n, decB.S.row_ptr, decB.S.col, decB.S.val, residue=rB)
    got = host(c.approx_matmul(dA, gpu(B), dB))
    assert rel(got, want) < TOL_F32


@pytest.mark.parametrize("m,n,nnz", [(8, 8, 0), (8, 8, 64), (37, 53, 100), (256, 256, 655), (1000, 300, 4000)])
def test_sparse_extract_exact(m, n, nnz):
    """Device extraction returns the oracle's CSR exactly (ties included)."""
    note(f"sparse extract m={m} n={n} nnz={nnz}")
    rng = np.random.default_rng(m + nnz)
    A = np.round(rng.standard_normal((m, n)) * 4) / 4   # many exact ties
    A = f32(A)
    want = osp.extract_dominant(A, nnz)
    c = ctx()
    d = c.decompose(gpu(A), "sparse", 0, sparse_nnz=nnz)
    rp, col, val = d.sparse_part()
    assert np.array_equal(rp, want.row_ptr)
    assert np.array_equal(col, want.col)
    assert np.array_equal(val.astype(np.float64), want.val)


def test_sparse_decompose_end_to_end():
    n = 256
    rng = np.random.default_rng(77)
    A = f32(inputs.spectral_matrix(n, n, inputs.decay_power(n, 1.5), rng))
    pos, vals = inputs.sparse_overlay(n, n, 0.01, 10.0, rng)
    A.reshape(-1)[pos] += vals
    A = f32(A)
    B = f32(rng.standard_normal((n, 64)))
    c = ctx()
    d = c.decompose(gpu(A), "sparse+tsvd", 16, sparse_frac=0.01)
    got = host(c.approx_matmul(d, gpu(B)))
    dec = osp.SparseDecomp(A, 0.01, "tsvd", 16)
    want = osp.apply_zeroth(dec, B)
    # same sparse set exactly, SVD of the residue by the randomized method
    rp, col, val = d.sparse_part()
    assert np.array_equal(col, dec.S.col)
    assert rel(got, want) < 1e-4


@pytest.mark.parametrize("n,ka,kb", [(128, 32, 32), (256, 32, 32), (512, 64, 32), (640, 32, 64), (1024, 64, 64), (384, 32, 0),
                                      (1280, 32, 32), (2048, 32, 0), (512, 128, 128), (768, 128, 0)])
def test_tsvd_split_path_first_order(n, ka, kb):
    """Shapes of the three-launch path (direct panels, reduction, output GEMM
    on split bfloat16 operands): float32 accuracy against the oracle.  Rank-32
    panels with n a multiple of 128 take the pipelined form (three load batches
    rotating per wave); n = 128 gives the H job a single batch, n = 1280 batch
    counts that are not multiples of three."""
    note(f"tsvd split path n={n} ka={ka} kb={kb}")
    sig = inputs.decay_power(n, 1.5)
    A = _spectral(n, n, sig, 21 + n)
    B = _spectral(n, n, sig, 22 + n)
    decA = ot.TSVDDecomp(A, ka)
    c = ctx()
    Ag, Bg = gpu(A), gpu(B)
    dA = c.import_tsvd(decA.U, decA.s, decA.V, A=Ag)
    if kb == 0:
        got = host(c.approx_matmul(dA, Bg))
        want = ot.apply_zeroth(decA, B)
    else:
        decB = ot.TSVDDecomp(B, kb)
        dB = c.import_tsvd(decB.U, decB.s, decB.V, A=Bg)
        got = host(c.approx_matmul(dA, Bg, dB))
        want = op.algorithm(decA, B, decB)
    assert rel(got, want) < TOL_F32


@pytest.mark.parametrize("m,n,p,k", [(128, 128, 128, 32), (384, 640, 256, 64), (256, 1024, 768, 32)])
def test_tsvd_split_path_zeroth_rect(m, n, p, k):
    note(f"tsvd split zeroth m={m} n={n} p={p} k={k}")
    rng = np.random.default_rng(m + n + p + k)
    A = _spectral(m, n, inputs.decay_power(min(m, n), 1.0), k + 1)
    B = f32(rng.standard_normal((n, p)))
    dec = ot.TSVDDecomp(A, k)
    c = ctx()
    d = c.import_tsvd(dec.U, dec.s, dec.V)
    assert rel(host(c.approx_matmul(d, gpu(B))), ot.apply_zeroth(dec, B)) < TOL_F32


def test_tsvd_first_order_full_size_sampled():
    """The benchmark's step at full size (n = 4096, rank 32 for A and B, the
    generator's exact leading factors imported), checked on sampled columns."""
    torch = torch_cuda()
    n, k = 4096, 32
    note("tsvd first order full size")
    sig = inputs.decay_power(n, 1.5)
    facs, mats = [], []
    for operand in (0, 1):
        rng = inputs.rng_of(2, operand)
        Q1 = inputs.haar_columns(n, n, rng, device="cuda")
        Q2 = inputs.haar_columns(n, n, rng, device="cuda")
        s64 = torch.from_numpy(sig).cuda()
        mats.append(((Q1 * s64) @ Q2.t()).float().contiguous())
        facs.append((Q1[:, :k].cpu().numpy(), sig[:k], Q2[:, :k].cpu().numpy()))
        del Q1, Q2
    A, B = mats
    c = ctx()
    dA = c.import_tsvd(*facs[0], A=A)
    dB = c.import_tsvd(*facs[1], A=B)
    out = c.approx_matmul(dA, B, dB)
    torch.cuda.synchronize()
    cols = np.sort(np.random.default_rng(9).choice(n, 24, replace=False))
    Ah = A.double().cpu().numpy()
    Bc = B[:, cols].double().cpu().numpy()
    UA, sA, VA = (f32(x) for x in facs[0])
    UB, sB, VB = (f32(x) for x in facs[1])
    decA = ot.TSVDDecomp(Ah, k, U=UA, s=sA, V=VA)
    Btil_c = (UB * sB[None, :]) @ VB[cols].T
    want = ot.apply_zeroth(decA, Bc) + decA.residual_dense() @ Btil_c
    got = out[:, cols].double().cpu().numpy()
    assert rel(got, want) < TOL_F32

"""Sparse path at n = 16384 (0.5 % Laplace(20) dominant entries over a
rank-1024 decay): extraction checked by properties that hold at any size, the
products S B and X S checked against the float64 oracle on sampled rows and
columns of the full-size launch."""
import numpy as np
import pytest

from oracle import sparse as osp
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, note, rel, torch_cuda

pytestmark = pytest.mark.gpu

N = 16384
FRAC = 0.005


@pytest.fixture(scope="module")
def c5():
    torch = torch_cuda()
    note(f"sparse large: generating n={N} operand")
    pair = inputs.workload_lowrank_sparse(N, device="cuda")
    A = pair.A.float().contiguous()
    del pair
    torch.cuda.empty_cache()
    c = ctx()
    d = c.decompose(A, "sparse", 0, sparse_frac=FRAC)
    rp, col, val = d.sparse_part()
    return {"A": A, "c": c, "d": d, "rp": rp, "col": col, "val": val}


def _sub_rows(rp, col, val, rows, n):
    """CSR of the given rows only (same entries, same order)."""
    srp = [0]
    scol, sval = [], []
    for r in rows:
        scol.extend(col[rp[r]:rp[r + 1]])
        sval.extend(val[rp[r]:rp[r + 1]])
        srp.append(len(scol))
    return osp.CSR(len(rows), n, np.array(srp), np.array(scol, dtype=np.int64), np.array(sval, dtype=np.float64))


def _sub_cols(rp, col, val, cols, m):
    """CSR restricted to the given columns, renumbered 0..len(cols)-1."""
    where = {int(c): i for i, c in enumerate(cols)}
    srp = [0]
    scol, sval = [], []
    for r in range(m):
        for e in range(rp[r], rp[r + 1]):
            j = where.get(int(col[e]))
            if j is not None:
                scol.append(j)
                sval.append(val[e])
        srp.append(len(scol))
    return osp.CSR(m, len(cols), np.array(srp), np.array(scol, dtype=np.int64), np.array(sval, dtype=np.float64))


def test_extract_large_properties(c5):
    A, rp, col, val = c5["A"], c5["rp"], c5["col"], c5["val"]
    note("sparse large: extraction properties")
    nnz = int(round(FRAC * N * N))
    assert rp[0] == 0 and rp[-1] == nnz and len(col) == nnz
    assert np.all(np.diff(rp) >= 0)
    thresh = float(np.min(np.abs(val)))
    rows = np.sort(np.random.default_rng(1).choice(N, 24, replace=False))
    Ah = A[rows].double().cpu().numpy()
    for i, r in enumerate(rows):
        cs = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(cs) > 0)
        assert np.array_equal(Ah[i, cs], val[rp[r]:rp[r + 1]].astype(np.float64))
        rest = np.delete(np.abs(Ah[i]), cs)
        assert rest.size == 0 or np.max(rest) <= thresh


def test_spmm_large_sampled(c5):
    torch = torch_cuda()
    c, d, rp, col, val = c5["c"], c5["d"], c5["rp"], c5["col"], c5["val"]
    note("sparse large: S B")
    g = torch.Generator(device="cuda")
    g.manual_seed(inputs.seed_of(5, 4))
    B = torch.randn((N, N), generator=g, device="cuda", dtype=torch.float32)
    out = c.approx_matmul(d, B)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    rows = np.sort(rng.choice(N, 16, replace=False))
    cols = np.sort(rng.choice(N, 16, replace=False))
    want = osp.spmm(_sub_rows(rp, col, val, rows, N), B[:, cols].double().cpu().numpy())
    got = out[rows][:, cols].double().cpu().numpy()
    assert rel(got, want) < TOL_F32


def test_dense_times_sparse_large_sampled(c5):
    """X S_B through the first-order term of an empty circulant truncation
    whose residual is X."""
    torch = torch_cuda()
    c, d, rp, col, val = c5["c"], c5["d"], c5["rp"], c5["col"], c5["val"]
    note("sparse large: X S")
    g = torch.Generator(device="cuda")
    g.manual_seed(inputs.seed_of(5, 5))
    X = torch.randn((N, N), generator=g, device="cuda", dtype=torch.float32)
    B = torch.zeros((N, N), device="cuda", dtype=torch.float32)
    dA = c.import_circulant(N, [], np.zeros((0, N)), residual=X)
    out = c.approx_matmul(dA, B, d)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(N, 8, replace=False))
    cols = np.sort(rng.choice(N, 24, replace=False))
    want = osp.dense_times_sparse(X[rows].double().cpu().numpy(), _sub_cols(rp, col, val, cols, N))
    got = out[rows][:, cols].double().cpu().numpy()
    assert rel(got, want) < TOL_F32


@pytest.mark.parametrize("m,n,p,nnz", [(5, 7, 3, 9), (64, 33, 130, 200), (300, 129, 67, 1000)])
def test_spmm_ragged(m, n, p, nnz):
    """Partial slices, rows not a multiple of the row group, p not a multiple
    of 4 (scalar path)."""
    torch = torch_cuda()
    note(f"sparse ragged S B m={m} n={n} p={p} nnz={nnz}")
    rng = np.random.default_rng(m + n + p)
    A = rng.standard_normal((m, n)).astype(np.float32).astype(np.float64)
    S = osp.extract_dominant(A, nnz)
    c = ctx()
    d = c.import_sparse(m, n, S.row_ptr, S.col, S.val)
    B = rng.standard_normal((n, p)).astype(np.float32).astype(np.float64)
    got = c.approx_matmul(d, torch.from_numpy(B.astype(np.float32)).cuda())
    assert rel(got.double().cpu().numpy(), osp.spmm(S, B)) < TOL_F32


@pytest.mark.parametrize("n,k,nnz", [(7, 2, 9), (129, 5, 700), (300, 9, 2000)])
def test_dense_times_sparse_ragged(n, k, nnz):
    """Atil B + Delta A S_B with a truncated-SVD left operand (Delta A from the
    borrowed A) and a sparse right operand, at sizes that leave partial tiles."""
    from oracle import tsvd as ot
    torch = torch_cuda()
    note(f"sparse ragged X S n={n} k={k} nnz={nnz}")
    rng = np.random.default_rng(n + k)
    X = rng.standard_normal((n, n)).astype(np.float32).astype(np.float64)
    Bm = rng.standard_normal((n, n)).astype(np.float32).astype(np.float64)
    S = osp.extract_dominant(Bm, nnz)
    decA = ot.TSVDDecomp(X, k)
    want = ot.apply_zeroth(decA, Bm) + osp.dense_times_sparse(decA.residual_dense(), S)
    c = ctx()
    Xg = torch.from_numpy(X.astype(np.float32)).cuda()
    dA = c.import_tsvd(decA.U, decA.s, decA.V, A=Xg)
    dB = c.import_sparse(n, n, S.row_ptr, S.col, S.val)
    got = c.approx_matmul(dA, torch.from_numpy(Bm.astype(np.float32)).cuda(), dB)
    assert rel(got.double().cpu().numpy(), want) < TOL_F32


def test_c5_first_order_identity_sampled():
    """The full first-order product of the n = 16384 workload (both operands
    decomposed on the device as S + circulant_64(R)) satisfies
    M1 = A B - Delta A Delta B (eq. (2.1)-(2.3)) on sampled columns, with
    Btil e_j and Atil (Delta B e_j) from the library's own zeroth-order
    products and everything else in float64."""
    torch = torch_cuda()
    note("sparse + circulant first-order identity")
    pair = inputs.workload_lowrank_sparse(N, device="cuda")
    A = pair.A.float().contiguous()
    B = pair.B.float().contiguous()
    del pair
    torch.cuda.empty_cache()
    c = ctx()
    dA = c.decompose(A, "sparse+circulant", 64, sparse_frac=FRAC)
    dB = c.decompose(B, "sparse+circulant", 64, sparse_frac=FRAC)
    M1 = c.approx_matmul(dA, B, dB)
    cols = torch.from_numpy(np.sort(np.random.default_rng(5).choice(N, 32, replace=False))).cuda()
    E = torch.zeros((N, len(cols)), device="cuda", dtype=torch.float32)
    E[cols, torch.arange(len(cols), device="cuda")] = 1.0
    Bhat = c.approx_matmul(dB, E)                   # Btil[:, cols]
    dBc = B[:, cols].double() - Bhat.double()      # Delta B[:, cols]
    AhatdB = c.approx_matmul(dA, dBc.float().contiguous()).double()
    A64 = A.double()
    want = A64 @ B[:, cols].double() - (A64 @ dBc - AhatdB)
    got = M1[:, cols].double()
    assert float((got - want).norm() / want.norm()) < TOL_F32


@pytest.mark.parametrize("m,n,p,nnz", [(700, 9000, 67, 20000), (333, 12289, 128, 9000), (100, 20000, 64, 8000),
                                       (129, 16385, 36, 4000)])
def test_spmm_blocked_inner(m, n, p, nnz):
    """Inner dimension above 8192: each row's entries are taken per block of
    4096 inner indices (the last block partial), later blocks accumulating."""
    torch = torch_cuda()
    note(f"sparse blocked S B m={m} n={n} p={p} nnz={nnz}")
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)).astype(np.float32).astype(np.float64)
    S = osp.extract_dominant(A, nnz)
    B = rng.standard_normal((n, p)).astype(np.float32).astype(np.float64)
    c = ctx()
    d = c.import_sparse(m, n, S.row_ptr, S.col, S.val)
    got = c.approx_matmul(d, torch.from_numpy(B.astype(np.float32)).cuda())
    assert rel(got.double().cpu().numpy(), osp.spmm(S, B)) < TOL_F32


def test_spmm_unsorted_rows_long_inner():
    """Rows stored with descending column indices keep the one-pass gather."""
    torch = torch_cuda()
    m, n, p, nnz = 200, 9000, 64, 6000
    note(f"sparse unsorted rows m={m} n={n}")
    rng = np.random.default_rng(17)
    A = rng.standard_normal((m, n)).astype(np.float32).astype(np.float64)
    S = osp.extract_dominant(A, nnz)
    col, val = S.col.copy(), S.val.copy()
    for i in range(m):
        a, b = S.row_ptr[i], S.row_ptr[i + 1]
        col[a:b] = col[a:b][::-1]
        val[a:b] = val[a:b][::-1]
    R = osp.CSR(m, n, S.row_ptr, col, val)
    B = rng.standard_normal((n, p)).astype(np.float32).astype(np.float64)
    c = ctx()
    d = c.import_sparse(m, n, R.row_ptr, R.col, R.val)
    got = c.approx_matmul(d, torch.from_numpy(B.astype(np.float32)).cuda())
    assert rel(got.double().cpu().numpy(), osp.spmm(R, B)) < TOL_F32


def test_dense_times_sparse_blocked_inner():
    """X S_B with 9000 inner indices (CSC columns taken per block of 4096 rows)
    through the first-order term of an empty circulant truncation whose
    residual is X; sampled rows against the oracle."""
    torch = torch_cuda()
    n, p, nnz = 9000, 96, 5000
    note(f"sparse blocked X S n={n} p={p}")
    rng = np.random.default_rng(23)
    Sd = rng.standard_normal((n, p)).astype(np.float32).astype(np.float64)
    S = osp.extract_dominant(Sd, nnz)
    g = torch.Generator(device="cuda")
    g.manual_seed(inputs.seed_of(5, 6))
    X = torch.randn((n, n), generator=g, device="cuda", dtype=torch.float32)
    c = ctx()
    dA = c.import_circulant(n, [], np.zeros((0, n)), residual=X)
    dB = c.import_sparse(n, p, S.row_ptr, S.col, S.val)
    out = c.approx_matmul(dA, torch.zeros((n, p), device="cuda", dtype=torch.float32), dB)
    torch.cuda.synchronize()
    rows = np.sort(rng.choice(n, 12, replace=False))
    want = osp.dense_times_sparse(X[rows].double().cpu().numpy(), S)
    assert rel(out[rows].double().cpu().numpy(), want) < TOL_F32

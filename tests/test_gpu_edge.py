"""Degenerate and boundary cases of the GPU path: empty products, rank 0,
zero and rank-deficient operands, the full circulant expansion (K = n gives A
back, Thm. 1.1), the full sparse part (f = 1 gives A back), 1 x 1 operands,
batch size limits."""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import sparse as osp
from oracle import tsvd as ot
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu


def test_empty_product_is_a_no_op():
    torch = torch_cuda()
    n = 64
    A = f32(inputs.spectral_matrix(n, n, inputs.decay_exp(n), np.random.default_rng(1)))
    c = ctx()
    dec = ot.TSVDDecomp(A, 8)
    d = c.import_tsvd(dec.U, dec.s, dec.V, A=gpu(A))
    B = torch.zeros((n, 0), device="cuda", dtype=torch.float32)
    out = c.approx_matmul(d, B)
    assert tuple(out.shape) == (n, 0)
    dc = c.import_circulant(n, [0], np.ones((1, n)))
    assert tuple(c.approx_matmul(dc, B).shape) == (n, 0)


def test_rank_zero_truncations_give_zero():
    n, p = 96, 40
    rng = np.random.default_rng(2)
    B = f32(rng.standard_normal((n, p)))
    c = ctx()
    A = gpu(rng.standard_normal((n, n)))
    d = c.decompose(A, "tsvd", 0)
    assert d.info()["K_eff"] == 0
    out = gpu(np.full((n, p), 5.0))
    assert np.all(host(c.approx_matmul(d, gpu(B), out=out)) == 0)


def test_zero_operand():
    """A = 0: no component survives (randomized SVD and circulant), products are 0."""
    n = 128
    c = ctx()
    Z = gpu(np.zeros((n, n)))
    B = gpu(np.random.default_rng(3).standard_normal((n, 16)))
    dt = c.decompose(Z, "tsvd", 8)
    assert dt.info()["K_eff"] == 0 and dt.info()["norm_A"] == 0
    assert np.all(host(c.approx_matmul(dt, B)) == 0)
    dcirc = c.decompose(Z, "circulant", 8)
    assert np.all(dcirc.energies() == 0)
    assert np.all(host(c.approx_matmul(dcirc, B)) == 0)


def test_rank_deficient_operand():
    """rank 3 < k = 8: the three singular values are found, the other five are
    at rounding level, and the product matches the exact one."""
    n, r, k = 256, 3, 8
    rng = np.random.default_rng(4)
    sig = np.array([3.0, 2.0, 1.0])
    A = f32(inputs.spectral_matrix(n, n, sig, rng))  # rank 3 before rounding
    c = ctx()
    d = c.decompose(gpu(A), "tsvd", k)
    U, s, V = d.tsvd_factors()
    assert np.allclose(s[:r], np.linalg.svd(A, compute_uv=False)[:r], rtol=1e-5)
    assert np.all(s[r:] < 1e-5 * s[0])
    B = f32(rng.standard_normal((n, 32)))
    assert rel(host(c.approx_matmul(d, gpu(B))), A @ B) < 1e-5


@pytest.mark.parametrize("n", [8, 64, 256])
def test_circulant_full_expansion_is_exact(n):
    """K = n keeps every component: Atil = A (Thm. 1.1) and the product is AB."""
    note(f"circulant K = n = {n}")
    rng = np.random.default_rng(n)
    A = f32(rng.standard_normal((n, n)))
    B = f32(rng.standard_normal((n, 24)))
    dec = oc.CirculantDecomp(A, n)
    assert len(dec.S) == n
    c = ctx()
    d = c.import_circulant(n, dec.S, dec.L)
    assert rel(host(c.approx_matmul(d, gpu(B))), A @ B) < TOL_F32
    dd = c.decompose(gpu(A), "circulant", n)
    assert dd.info()["K_eff"] == n
    assert rel(host(c.approx_matmul(dd, gpu(B))), A @ B) < TOL_F32


def test_sparse_full_part_is_exact():
    """f = 1: S = A, the residue is zero (its truncation has no component), SB = AB."""
    n = 128
    rng = np.random.default_rng(6)
    A = f32(rng.standard_normal((n, n)))
    B = f32(rng.standard_normal((n, 20)))
    c = ctx()
    d = c.decompose(gpu(A), "sparse+tsvd", 4, sparse_frac=1.0)
    assert d.info()["nnz"] == n * n
    assert rel(host(c.approx_matmul(d, gpu(B))), A @ B) < TOL_F32


def test_one_by_one():
    c = ctx()
    A = np.array([[2.5]])
    B = np.array([[-4.0, 0.5, 3.0]])
    dec = ot.TSVDDecomp(A, 1)
    d = c.import_tsvd(dec.U, dec.s, dec.V)
    assert rel(host(c.approx_matmul(d, gpu(B))), A @ B) < TOL_F32
    ds = c.import_sparse(1, 1, [0, 1], [0], [2.5])
    assert rel(host(c.approx_matmul(ds, gpu(B))), A @ B) < TOL_F32


def test_batch_size_limits():
    from paper_2504_19308_amd import AmmError
    torch = torch_cuda()
    c = ctx()
    rng = np.random.default_rng(7)
    A = f32(inputs.spectral_matrix(128, 128, inputs.decay_power(128, 1.0), rng))
    dec = ot.TSVDDecomp(A, 16)
    d = c.import_tsvd(dec.U, dec.s, dec.V)
    B = torch.from_numpy(f32(rng.standard_normal((128, 128))).astype(np.float32)).cuda()
    want = ot.apply_zeroth(dec, host(B))
    plan = c.batch_plan([d] * 256, [B] * 256)     # the maximum entry count, all sharing B
    outs = plan.run(use_graph=True)
    torch.cuda.synchronize()
    for o in outs[::51]:
        assert rel(host(o), want) < TOL_F32
    with pytest.raises(AmmError):
        c.batch_plan([d] * 257, [B] * 257)

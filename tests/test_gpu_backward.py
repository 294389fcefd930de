"""GPU backward of the approximate product (frozen truncation structure)
against the float64 oracle's backward, which the CPU suite pins with central
finite differences.  Bar: 1e-5 relative Frobenius per gradient."""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import product as op
from oracle import sparse as osp
from oracle import tsvd as ot
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu


def _w(n, alpha, seed):
    return f32(inputs.spectral_matrix(n, n, inputs.decay_power(n, alpha), np.random.default_rng(seed)))


@pytest.mark.parametrize("n,p,k", [(64, 40, 8), (256, 256, 16), (512, 384, 32), (1024, 2048, 128), (300, 70, 7)])
def test_backward_tsvd(n, p, k):
    note(f"backward tsvd n={n} p={p} k={k}")
    rng = np.random.default_rng(n + p)
    W = _w(n, 1.2, n)
    X = f32(rng.standard_normal((n, p)))
    dY = f32(rng.standard_normal((n, p)))
    dec = ot.TSVDDecomp(W, k)
    want_dx, want_dw = op.backward(dec, X, dY)
    c = ctx()
    d = c.import_tsvd(dec.U, dec.s, dec.V)
    dX, dW = c.approx_matmul_backward(d, gpu(X), gpu(dY))
    assert rel(host(dX), want_dx) < TOL_F32
    assert rel(host(dW), want_dw) < TOL_F32


@pytest.mark.parametrize("n,p,K", [(16, 8, 3), (64, 64, 9), (256, 100, 16), (1024, 256, 33), (300, 64, 11), (700, 20, 5)])
def test_backward_circulant(n, p, K):
    note(f"backward circulant n={n} p={p} K={K}")
    rng = np.random.default_rng(n + K)
    W = f32(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    X = f32(rng.standard_normal((n, p)))
    dY = f32(rng.standard_normal((n, p)))
    dec = oc.CirculantDecomp(W, K)
    want_dx, want_dw = op.backward(dec, X, dY)
    c = ctx()
    d = c.import_circulant(n, dec.S, dec.L)
    dX, dW = c.approx_matmul_backward(d, gpu(X), gpu(dY))
    assert rel(host(dX), want_dx) < TOL_F32
    assert rel(host(dW), want_dw) < TOL_F32


@pytest.mark.parametrize("n,p,frac", [(64, 32, 0.05), (256, 128, 0.01)])
def test_backward_sparse_tsvd(n, p, frac):
    rng = np.random.default_rng(n)
    W = _w(n, 1.5, n + 1)
    pos, vals = inputs.sparse_overlay(n, n, frac, 10.0, rng)
    W.reshape(-1)[pos] += vals
    W = f32(W)
    X = f32(rng.standard_normal((n, p)))
    dY = f32(rng.standard_normal((n, p)))
    dec = osp.SparseDecomp(W, frac, "tsvd", 6)
    want_dx, want_dw = op.backward(dec, X, dY)
    c = ctx()
    r = c.import_tsvd(dec.inner.U, dec.inner.s, dec.inner.V)
    d = c.import_sparse(n, n, dec.S.row_ptr, dec.S.col, dec.S.val, residue=r)
    dX, dW = c.approx_matmul_backward(d, gpu(X), gpu(dY))
    assert rel(host(dX), want_dx) < TOL_F32
    assert rel(host(dW), want_dw) < TOL_F32


def test_autograd_function_matches_oracle():
    """torch.autograd through the library: loss = <Wtil X, G>."""
    torch = torch_cuda()
    from paper_2504_19308_amd import approx_linear
    n, p, k = 256, 128, 16
    rng = np.random.default_rng(3)
    Wh = _w(n, 1.2, 5)
    Xh = f32(rng.standard_normal((n, p)))
    Gh = f32(rng.standard_normal((n, p)))
    dec = ot.TSVDDecomp(Wh, k)
    c = ctx()
    d = c.import_tsvd(dec.U, dec.s, dec.V)
    W = gpu(Wh).requires_grad_(True)
    X = gpu(Xh).requires_grad_(True)
    Y = approx_linear(W, X, c, d)
    loss = (Y * gpu(Gh)).sum()
    loss.backward()
    want_dx, want_dw = op.backward(dec, Xh, Gh)
    assert rel(host(X.grad), want_dx) < TOL_F32
    assert rel(host(W.grad), want_dw) < TOL_F32
    assert rel(host(Y.detach()), ot.apply_zeroth(dec, Xh)) < TOL_F32


def test_backward_full_size_tsvd_sampled():
    """W 4096 x 4096 (sigma_i = i^-1.2), X 4096 x 8192 as in the layer
    workload; dX checked on sampled columns, dW on sampled rows."""
    torch = torch_cuda()
    n, p, k = 4096, 8192, 128
    rng = np.random.default_rng(11)
    Wg = inputs.spectral_matrix(n, n, inputs.decay_power(n, 1.2), rng, device="cuda").float()
    Xg = torch.from_numpy(rng.standard_normal((n, p)).astype(np.float32)).cuda()
    dYg = torch.from_numpy(rng.standard_normal((n, p)).astype(np.float32)).cuda()
    c = ctx()
    d = c.decompose(Wg, "tsvd", k, seed=4)
    U, s, V = d.tsvd_factors()
    dX, dW = c.approx_matmul_backward(d, Xg, dYg)
    torch.cuda.synchronize()
    U64, s64, V64 = U.astype(np.float64), s.astype(np.float64), V.astype(np.float64)
    cols = np.sort(rng.choice(p, 32, replace=False))
    dYc = dYg[:, cols].double().cpu().numpy()
    want_dx = (V64 * s64) @ (U64.T @ dYc)
    assert rel(dX[:, cols].double().cpu().numpy(), want_dx) < TOL_F32
    rows = np.sort(rng.choice(n, 16, replace=False))
    Gy = U64.T @ dYg.double().cpu().numpy()
    Gx = V64.T @ Xg.double().cpu().numpy()
    want_dw_rows = (U64[rows] @ (Gy @ Gx.T)) @ V64.T
    assert rel(dW[rows].double().cpu().numpy(), want_dw_rows) < TOL_F32

"""Operands with row pitches (amm_approx_matmul_strided): B and out as column
panels of larger row-major matrices.  Every kind gives the product of the
packed operands (the circulant and sparse + circulant zeroth-order products
read and write at the pitches; the others through packed copies), the
columns outside the panels stay untouched, and bad pitches or overlapping
operands are refused."""
import ctypes as C

import numpy as np
import pytest

from oracle import circulant as oc
from paper_2504_19308_amd import AmmError, _lib, inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu


def _panel_product(c, dA, B, dB, m, c0=8, o0=20, extra=36):
    """B placed at columns c0.. of a wider matrix, out at columns o0.. of
    another (filled with a sentinel); returns (panel result, wide out)."""
    torch = torch_cuda()
    n, p = B.shape
    Bw = torch.randn((n, p + extra), device="cuda")
    Bw[:, c0:c0 + p] = B
    Ow = torch.full((m, p + extra), 7.25, device="cuda")
    got = c.approx_matmul(dA, Bw[:, c0:c0 + p], dB, out=Ow[:, o0:o0 + p])
    torch.cuda.synchronize()
    return got, Ow


def _untouched(Ow, o0, p):
    w = host(Ow)
    keep = np.ones(w.shape[1], dtype=bool)
    keep[o0:o0 + p] = False
    return bool(np.all(w[:, keep] == 7.25))


@pytest.mark.parametrize("kind,n,K,p,extra", [
    ("circulant", 1024, 8, 40, {}),                 # read and written at the pitches
    ("circulant", 4096, 16, 64, {"spectral_fp16": True}),
    ("circulant", 1000, 6, 24, {}),                 # chirp path: packed copies
    ("tsvd", 512, 32, 128, {}),
    ("sparse+circulant", 1024, 8, 64, {"sparse_frac": 0.01}),   # at the pitches
    ("sparse+tsvd", 512, 16, 48, {"sparse_frac": 0.02}),
    ("sfft", 512, 8, 32, {}),
])
def test_strided_zeroth_matches_packed(kind, n, K, p, extra):
    torch = torch_cuda()
    note(f"strided zeroth {kind} n={n} K={K} p={p} {extra}")
    rng = np.random.default_rng(n + K + p)
    A = gpu(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    B = gpu(rng.standard_normal((n, p)))
    c = ctx()
    d = c.decompose(A, kind, K, **extra)
    want = c.approx_matmul(d, B)
    got, Ow = _panel_product(c, d, B, None, n)
    assert rel(host(got), host(want)) < 1e-6
    assert _untouched(Ow, 20, p)
    if kind == "circulant" and not extra:
        o = oc.CirculantDecomp(host(A), K)
        assert list(d.frequencies()) == list(o.S)
        assert rel(host(got), np.real(oc.apply_zeroth(o, host(B)))) < TOL_F32


@pytest.mark.parametrize("kind,n,K", [("circulant", 1024, 8), ("tsvd", 512, 32), ("sparse+circulant", 1024, 8)])
def test_strided_first_order_matches_packed(kind, n, K):
    torch = torch_cuda()
    note(f"strided first order {kind} n={n} K={K}")
    rng = np.random.default_rng(n + 3 * K)
    A = gpu(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    B = gpu(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    extra = {"sparse_frac": 0.01} if kind.startswith("sparse") else {}
    c = ctx()
    dA = c.decompose(A, kind, K, keep_residual=True, **extra)
    dB = c.decompose(B, kind, K, keep_residual=True, **extra)
    want = c.approx_matmul(dA, B, dB)
    got, Ow = _panel_product(c, dA, B, dB, n, extra=20)
    assert rel(host(got), host(want)) < 1e-6
    assert _untouched(Ow, 20, n)


def test_strided_unaligned_sparse_uses_packed_copies():
    """A pitch that is not a multiple of 4 on the sparse + circulant path."""
    torch = torch_cuda()
    n, p = 1024, 30
    rng = np.random.default_rng(17)
    A = gpu(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    B = gpu(rng.standard_normal((n, p)))
    c = ctx()
    d = c.decompose(A, "sparse+circulant", 8, sparse_frac=0.01)
    want = c.approx_matmul(d, B)
    got, Ow = _panel_product(c, d, B, None, n, c0=3, o0=5, extra=7)
    assert rel(host(got), host(want)) < 1e-6
    assert _untouched(Ow, 5, p)


def test_strided_refusals():
    torch = torch_cuda()
    n, p = 256, 16
    rng = np.random.default_rng(2)
    A = gpu(inputs.toeplitz_uniform(n, rng))
    c = ctx()
    d = c.decompose(A, "circulant", 4)
    lib = _lib.load()
    W = torch.zeros((n + 1, 64), device="cuda")     # one spare row: panels that run past column 64 stay inside
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ptr = lambda t, off=0: C.c_void_p(t.data_ptr() + 4 * off)
    assert lib.amm_approx_matmul_strided(c.handle, d.handle, None, ptr(W), n, p, p - 1, ptr(W, 32), 64, s) == 2
    assert lib.amm_approx_matmul_strided(c.handle, d.handle, None, ptr(W), n, p, 64, ptr(W, 32), p - 1, s) == 2
    # panels of one matrix that share columns: refused; side by side: accepted
    assert lib.amm_approx_matmul_strided(c.handle, d.handle, None, ptr(W), n, p, 64, ptr(W, 8), 64, s) == 1
    # B's rows run 8 floats into the next row, where out's panel starts at column 4
    assert lib.amm_approx_matmul_strided(c.handle, d.handle, None, ptr(W, 56), n, p, 64, ptr(W, 64 + 4), 64, s) == 1
    assert lib.amm_approx_matmul_strided(c.handle, d.handle, None, ptr(W), n, 0, 64, ptr(W, 16), 64, s) == 0
    W[:n, :p] = gpu(rng.standard_normal((n, p)))
    assert lib.amm_approx_matmul_strided(c.handle, d.handle, None, ptr(W), n, p, 64, ptr(W, 16), 64, s) == 0
    torch.cuda.synchronize()
    assert rel(host(W[:n, 16:16 + p]), host(c.approx_matmul(d, W[:n, :p].contiguous()))) < 1e-6

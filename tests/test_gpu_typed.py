"""Described operands of any element type (amm_approx_matmul_ex and
amm_approx_matmul_backward_ex): bfloat16 and float16 inputs are widened
exactly, so the products equal the float32 products of the widened values
bit for bit; 16-bit outputs are those float32 results rounded once to
nearest even (torch's conversion rounds the same way).  One case is also
checked against the float64 oracle on the bfloat16-rounded operand."""
import ctypes as C

import numpy as np
import pytest

from oracle import circulant as oc
from paper_2504_19308_amd import _lib, inputs
from tests._gpu_common import TOL_F32, bf16, ctx, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu


def _dec(c, kind, n, K, rng):
    A = gpu(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    extra = {"sparse_frac": 0.01} if kind.startswith("sparse") else {}
    return A, c.decompose(A, kind, K, **extra)


@pytest.mark.parametrize("kind,n,K,p", [("circulant", 1024, 8, 48), ("tsvd", 512, 32, 64),
                                        ("sparse+circulant", 1024, 8, 40), ("circulant", 700, 6, 20)])
@pytest.mark.parametrize("dtype", ["bfloat16", "float16"])
def test_typed_inputs_and_outputs(kind, n, K, p, dtype):
    torch = torch_cuda()
    note(f"typed {kind} n={n} K={K} p={p} {dtype}")
    dt = getattr(torch, dtype)
    rng = np.random.default_rng(n + p)
    c = ctx()
    A, d = _dec(c, kind, n, K, rng)
    B16 = gpu(rng.standard_normal((n, p))).to(dt)
    want = c.approx_matmul(d, B16.float())                 # float32 product of the widened values
    got32 = c.approx_matmul(d, B16, out=torch.empty((n, p), device="cuda"))
    got16 = c.approx_matmul(d, B16)                        # out in B's type
    torch.cuda.synchronize()
    assert got16.dtype == dt
    assert torch.equal(got32, want)
    assert torch.equal(got16, want.to(dt))
    # a 16-bit column panel in, a float32 panel out
    W = torch.zeros((n, p + 10), dtype=dt, device="cuda")
    W[:, 3:3 + p] = B16
    O = torch.full((n, p + 6), 5.0, device="cuda")
    c.approx_matmul(d, W[:, 3:3 + p], out=O[:, 2:2 + p])
    torch.cuda.synchronize()
    assert torch.equal(O[:, 2:2 + p], want)
    assert bool((O[:, :2] == 5.0).all() and (O[:, 2 + p:] == 5.0).all())


def test_typed_against_oracle():
    torch = torch_cuda()
    n, K, p = 2048, 12, 32
    rng = np.random.default_rng(9)
    Ah = inputs.toeplitz_uniform(n, rng) + 0.05 * rng.standard_normal((n, n))
    Ah = np.asarray(Ah, dtype=np.float32).astype(np.float64)
    Bh = bf16(rng.standard_normal((n, p)))
    c = ctx()
    d = c.decompose(gpu(Ah), "circulant", K)
    o = oc.CirculantDecomp(Ah, K)
    assert list(d.frequencies()) == list(o.S)
    got = host(c.approx_matmul(d, gpu(Bh).bfloat16(), out=torch.empty((n, p), device="cuda")))
    assert rel(got, np.real(oc.apply_zeroth(o, Bh))) < TOL_F32


@pytest.mark.parametrize("kind,n,K", [("tsvd", 512, 32), ("circulant", 1024, 8), ("sparse+tsvd", 512, 16)])
def test_typed_backward(kind, n, K):
    torch = torch_cuda()
    note(f"typed backward {kind} n={n} K={K}")
    rng = np.random.default_rng(3 * n + K)
    c = ctx()
    A, d = _dec(c, kind, n, K, rng)
    p = 64
    X = gpu(rng.standard_normal((n, p))).bfloat16()
    dY = gpu(rng.standard_normal((n, p))).bfloat16()
    dX32, dW32 = c.approx_matmul_backward(d, X.float(), dY.float())
    dX, dW = c.approx_matmul_backward(d, X, dY)
    torch.cuda.synchronize()
    assert dX.dtype == torch.bfloat16 and dW.dtype == torch.float32
    assert torch.equal(dX, dX32.bfloat16())
    assert torch.equal(dW, dW32)


def test_typed_refusals():
    torch = torch_cuda()
    n = 256
    rng = np.random.default_rng(1)
    c = ctx()
    A, d = _dec(c, "circulant", n, 4, rng)
    lib = _lib.load()
    B = torch.zeros((n, 8), dtype=torch.bfloat16, device="cuda")
    O = torch.zeros((n, 8), device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    mb = _lib.AmmMatrix(C.c_void_p(B.data_ptr()), n, 8, 8, 7)                    # unknown element type
    mo = _lib.AmmMatrix(C.c_void_p(O.data_ptr()), n, 8, 8, _lib.AMM_F32)
    assert lib.amm_approx_matmul_ex(c.handle, d.handle, None, C.byref(mb), C.byref(mo), s) == 1
    mb = _lib.AmmMatrix(C.c_void_p(B.data_ptr()), n - 1, 8, 8, _lib.AMM_BF16)     # rows != n
    assert lib.amm_approx_matmul_ex(c.handle, d.handle, None, C.byref(mb), C.byref(mo), s) == 2
    mb = _lib.AmmMatrix(C.c_void_p(B.data_ptr()), n, 8, 4, _lib.AMM_BF16)         # pitch below the columns
    assert lib.amm_approx_matmul_ex(c.handle, d.handle, None, C.byref(mb), C.byref(mo), s) == 2
    mb = _lib.AmmMatrix(C.c_void_p(O.data_ptr()), n, 8, 8, _lib.AMM_BF16)         # out overlaps B
    assert lib.amm_approx_matmul_ex(c.handle, d.handle, None, C.byref(mb), C.byref(mo), s) == 1

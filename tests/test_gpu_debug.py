"""Debug mode (amm_ctx_set_debug, or AMM_DEBUG at context creation): matrix
pointers are checked to be device memory before anything is launched, and
every call synchronises its stream.  Host pointers are only ever passed
with zero columns or rows, so no kernel could read them even if a check
failed to refuse."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_2504_19308_amd import Context, inputs
from paper_2504_19308_amd import _lib
from tests._gpu_common import ctx, gpu, torch_cuda

pytestmark = pytest.mark.gpu


def _host_ptr(a):
    return C.c_void_p(a.ctypes.data)


def test_debug_refuses_host_pointers_before_launch():
    torch = torch_cuda()
    n = 256
    rng = np.random.default_rng(1)
    c = ctx()
    d = c.decompose(gpu(inputs.toeplitz_uniform(n, rng)), "circulant", 4)
    lib = _lib.load()
    host = np.zeros((n, 8), dtype=np.float32)
    out = torch.zeros((n, 8), device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # zero columns: nothing is read either way; only the debug check can object
    assert lib.amm_approx_matmul(c.handle, d.handle, None, _host_ptr(host), n, 0, C.c_void_p(out.data_ptr()), s) == 0
    c.set_debug(True)
    assert lib.amm_approx_matmul(c.handle, d.handle, None, _host_ptr(host), n, 0, C.c_void_p(out.data_ptr()), s) == 1
    assert b"not device memory" in lib.amm_last_error()
    assert lib.amm_approx_matmul(c.handle, d.handle, None, C.c_void_p(out.data_ptr()), n, 0, _host_ptr(host), s) == 1
    # decomposition of an empty operand: the body refuses the shape, the debug check the pointer first
    h = C.c_void_p()
    opts = _lib.AmmOpts()
    lib.amm_opts_default(C.byref(opts))
    assert lib.amm_decompose(c.handle, _host_ptr(host), 0, 0, 1, 4, C.byref(opts), s, C.byref(h)) == 1
    c.set_debug(False)
    assert lib.amm_decompose(c.handle, _host_ptr(host), 0, 0, 1, 4, C.byref(opts), s, C.byref(h)) == 2


def test_debug_products_unchanged():
    torch = torch_cuda()
    n, p = 1024, 32
    rng = np.random.default_rng(2)
    A = gpu(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    B = gpu(rng.standard_normal((n, p)))
    c = ctx()
    for kind in ("circulant", "tsvd", "sparse+circulant"):
        d = c.decompose(A, kind, 8, sparse_frac=0.01) if kind.startswith("sparse") else c.decompose(A, kind, 8)
        want = c.approx_matmul(d, B)
        c.set_debug(True)
        got = c.approx_matmul(d, B)
        dX, dW = c.approx_matmul_backward(d, B, B)
        c.set_debug(False)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        assert torch.isfinite(dX).all() and torch.isfinite(dW).all()


def test_debug_from_environment():
    torch = torch_cuda()
    n = 256
    rng = np.random.default_rng(3)
    old = os.environ.get("AMM_DEBUG")
    os.environ["AMM_DEBUG"] = "1"
    try:
        c = Context(0)
    finally:
        if old is None:
            del os.environ["AMM_DEBUG"]
        else:
            os.environ["AMM_DEBUG"] = old
    d = c.decompose(gpu(inputs.toeplitz_uniform(n, rng)), "circulant", 4)
    lib = _lib.load()
    host = np.zeros((n, 4), dtype=np.float32)
    out = torch.zeros((n, 4), device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.amm_approx_matmul(c.handle, d.handle, None, _host_ptr(host), n, 0, C.c_void_p(out.data_ptr()), s) == 1

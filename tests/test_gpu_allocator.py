"""Caller-supplied device allocator (amm_ctx_create_with_allocator): every
device buffer of the context, its handles and its plans comes from the
caller's functions and goes back through them; products equal those of a
context that uses hipMalloc; a refusing allocator turns into AMM_ENOMEM."""
import numpy as np
import pytest

from paper_2504_19308_amd import AmmError, Context, inputs
from tests._gpu_common import ctx, gpu, note, torch_cuda

pytestmark = pytest.mark.gpu


class _Counting:
    """torch's caching allocator (current stream), with the live set kept."""

    def __init__(self, refuse=False):
        self.torch = torch_cuda()
        self.live, self.calls, self.frees, self.refuse = {}, 0, 0, refuse

    def alloc(self, nbytes, dev):
        self.calls += 1
        if self.refuse:
            return 0
        ptr = self.torch.cuda.caching_allocator_alloc(nbytes, dev)
        self.live[ptr] = nbytes
        return ptr

    def free(self, ptr, nbytes, dev):
        assert self.live.pop(ptr) == nbytes    # freed once, with its own size
        self.frees += 1
        self.torch.cuda.caching_allocator_delete(ptr)


@pytest.mark.parametrize("kind,n,K,extra", [
    ("circulant", 1024, 8, {}),
    ("circulant", 2048, 6, {"spectral_fp16": True}),
    ("tsvd", 512, 32, {}),
    ("sparse+circulant", 1024, 8, {"sparse_frac": 0.01}),
])
def test_allocator_products_and_balance(kind, n, K, extra):
    torch = torch_cuda()
    note(f"caller allocator {kind} n={n} K={K} {extra}")
    rng = np.random.default_rng(n + K)
    A = gpu(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    B = gpu(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    ref = ctx()
    rA = ref.decompose(A, kind, K, **extra)
    rB = ref.decompose(B, kind, K, **extra)
    blobA, blobB = rA.export(), rB.export()

    al = _Counting()
    base = torch.cuda.memory_allocated()
    c = Context(0, allocator=(al.alloc, al.free))
    # the same decomposition rebuilt on the caller's memory: identical products
    iA, iB = c.import_blob(blobA, A=A), c.import_blob(blobB, A=B)
    for d1, i1, d2, i2 in ((rA, iA, None, None), (rA, iA, rB, iB)):
        want = ref.approx_matmul(d1, B, d2)
        got = c.approx_matmul(i1, B, i2)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
    # decomposing on the device through the caller's memory
    dA = c.decompose(A, kind, K, **extra)
    got = c.approx_matmul(dA, B)
    want = ref.approx_matmul(rA, B)
    torch.cuda.synchronize()
    assert torch.allclose(got, want, rtol=1e-4, atol=1e-4 * float(want.abs().max()))
    assert al.calls > 0 and len(al.live) > 0
    held = sum(al.live.values())
    assert torch.cuda.memory_allocated() - base >= held
    note(f"  {al.calls} allocations, {len(al.live)} live ({held} bytes)")
    for d in (iA, iB, dA):
        d.close()
    c.close()
    torch.cuda.synchronize()
    assert al.live == {} and al.frees == al.calls


def test_allocator_torch_shorthand_and_batch_plan():
    torch = torch_cuda()
    n = 1024
    rng = np.random.default_rng(4)
    A = gpu(inputs.toeplitz_uniform(n, rng))
    Bs = [gpu(rng.standard_normal((n, 16))) for _ in range(3)]
    ref = ctx()
    c = Context(0, allocator="torch")
    blob = ref.decompose(A, "circulant", 8).export()
    d = c.import_blob(blob, A=A)
    plan = c.batch_plan([d] * 3, Bs)
    for graph in (False, True, True):
        outs = plan.run(use_graph=graph)
        torch.cuda.synchronize()
        for B, o in zip(Bs, outs):
            want = c.approx_matmul(d, B)
            torch.cuda.synchronize()
            assert torch.allclose(o, want, rtol=1e-5, atol=1e-5 * float(want.abs().max()))
    plan.close()
    d.close()
    c.close()


def test_allocator_refusal_is_enomem():
    torch = torch_cuda()
    n = 1024
    rng = np.random.default_rng(8)
    A = gpu(inputs.toeplitz_uniform(n, rng))
    al = _Counting(refuse=True)
    c = Context(0, allocator=(al.alloc, al.free))
    with pytest.raises(AmmError) as e:
        c.decompose(A, "circulant", 8)
    assert e.value.status == 4     # AMM_ENOMEM
    assert al.calls >= 1 and al.live == {}
    # the context stays usable once the allocator gives memory again
    al.refuse = False
    d = c.decompose(A, "circulant", 8)
    B = gpu(rng.standard_normal((n, 8)))
    got = c.approx_matmul(d, B)
    torch.cuda.synchronize()
    assert torch.isfinite(got).all()
    d.close()
    c.close()
    assert al.live == {}

"""Export / import of decomposition handles through the C ABI: a handle made
on the device, written to a host blob and rebuilt, gives the same products
bit for bit (zeroth and first order), for every decomposition kind; malformed
blobs are refused."""
import numpy as np
import pytest

from paper_2504_19308_amd import AmmError, inputs
from tests._gpu_common import ctx, gpu, note, torch_cuda

pytestmark = pytest.mark.gpu


def _same(x, y):
    torch = torch_cuda()
    return bool(torch.equal(x, y))


def _same_info(a, b):
    """Field by field, NaN equal to NaN (statistics a kind does not carry)."""
    for k in a:
        x, y = a[k], b[k]
        if isinstance(x, float) and np.isnan(x):
            if not np.isnan(y):
                return False
        elif x != y:
            return False
    return a.keys() == b.keys()


def _roundtrip(c, d, A=None):
    blob = d.export()
    assert blob[:4] == b"AMMX"
    return c.import_blob(blob, A=A), len(blob)


@pytest.mark.parametrize("kind,n,K,extra", [
    ("circulant", 512, 8, {}),
    ("circulant", 1024, 12, {"spectral_fp16": True}),
    ("tsvd", 512, 32, {}),
    ("sparse+circulant", 1024, 8, {"sparse_frac": 0.01}),
    ("sparse+tsvd", 512, 16, {"sparse_frac": 0.02}),
])
def test_roundtrip_products_identical(kind, n, K, extra):
    torch = torch_cuda()
    note(f"export round trip {kind} n={n} K={K} {extra}")
    rng = np.random.default_rng(n + K)
    A = gpu(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    B = gpu(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    c = ctx()
    dA = c.decompose(A, kind, K, **extra)
    dB = c.decompose(B, kind, K, **extra)
    iA, size = _roundtrip(c, dA, A=A)
    iB, _ = _roundtrip(c, dB, A=B)
    note(f"  blob {size} bytes")
    assert _same_info(iA.info(), dA.info())
    for d1, i1, d2, i2 in ((dA, iA, None, None), (dA, iA, dB, iB)):
        want = c.approx_matmul(d1, B, d2)
        got = c.approx_matmul(i1, B, i2)
        torch.cuda.synchronize()
        assert _same(got, want)


def test_roundtrip_blocked_and_sfft():
    torch = torch_cuda()
    c = ctx()
    rng = np.random.default_rng(9)
    A = gpu(rng.standard_normal((300, 128)))
    B = gpu(rng.standard_normal((128, 40)))
    d = c.decompose(A, "circulant", 6)
    i, _ = _roundtrip(c, d)
    assert i.info()["blocks"] == d.info()["blocks"] == 3
    assert _same(c.approx_matmul(i, B), c.approx_matmul(d, B))
    n = 256
    As = gpu(inputs.sinusoid_rows(n, n, np.random.default_rng(1)))
    Bs = gpu(inputs.sinusoid_rows(n, n, np.random.default_rng(2)).T.copy())
    ds = c.decompose(As, "sfft", 8)
    db = c.decompose(Bs, "sfft", 8)
    i1, _ = _roundtrip(c, ds)
    i2, _ = _roundtrip(c, db)
    assert _same(c.approx_matmul(i1, Bs, i2), c.approx_matmul(ds, Bs, db))
    torch.cuda.synchronize()


def test_import_refuses_malformed():
    c = ctx()
    rng = np.random.default_rng(3)
    A = gpu(rng.standard_normal((64, 64)))
    blob = c.decompose(A, "circulant", 4).export()
    with pytest.raises(AmmError, match="AMM_EINVAL"):
        c.import_blob(blob[:-1])
    with pytest.raises(AmmError, match="AMM_EINVAL"):
        c.import_blob(b"XXXX" + blob[4:])
    with pytest.raises(AmmError, match="AMM_EINVAL"):
        c.import_blob(blob[:40])

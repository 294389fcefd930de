"""The product entry point that allocates nothing (amm_approx_matmul_static):
its output against amm_approx_matmul's on the same handles and inputs, on two
calls in a row (the second smaller), zeroth and first order, through the C
ABI; and its refusals (other handle kinds, a need above the fixed array)."""
import numpy as np
import pytest

from paper_2504_19308_amd import AmmError, inputs
from tests._gpu_common import TOL_F32, ctx, note, torch_cuda

pytestmark = pytest.mark.gpu


def _operands(torch, m, n, p, seed):
    rng = np.random.default_rng(seed)
    A = torch.from_numpy(inputs.spectral_matrix(m, n, inputs.decay_power(min(m, n), 1.5), rng)).float().cuda()
    B = torch.from_numpy(inputs.spectral_matrix(n, p, inputs.decay_power(min(n, p), 1.5), rng)).float().cuda()
    return A.contiguous(), B.contiguous()


def _rel(x, y):
    return float((x.double() - y.double()).norm() / y.double().norm())


def test_static_matches_regular_two_calls():
    torch = torch_cuda()
    c = ctx()
    for (m, n, p, k, seed) in ((4096, 4096, 4096, 32, 1), (1024, 512, 256, 32, 2)):
        note(f"static product m={m} n={n} p={p} k={k}")
        A, B = _operands(torch, m, n, p, seed)
        dA = c.decompose(A, "tsvd", k, seed=seed)
        dB = c.decompose(B, "tsvd", k, seed=seed + 10)
        for dB_ in (None, dB):
            ref = c.approx_matmul(dA, B, dB_)
            out = torch.full_like(ref, float("nan"))
            c.approx_matmul_static(dA, B, out, dB_)
            torch.cuda.synchronize()
            assert torch.isfinite(out).all()
            err = _rel(out, ref)
            note(f"  {'first' if dB_ is not None else 'zeroth'} order: rel diff {err:.2e}")
            assert err <= TOL_F32


def test_static_refusals():
    torch = torch_cuda()
    c = ctx()
    A, B = _operands(torch, 256, 256, 256, 3)
    dc = c.decompose(A, "circulant", 8)
    out = torch.empty((256, 256), device="cuda")
    with pytest.raises(AmmError, match="AMM_EUNSUPPORTED"):
        c.approx_matmul_static(dc, B, out)
    d16 = c.decompose(A, "tsvd", 16)       # rank 16 has no split path
    with pytest.raises(AmmError, match="AMM_EUNSUPPORTED"):
        c.approx_matmul_static(d16, B, out)
    # rank 128 over 65536 output columns needs at least 2 x 128 x 65536 floats,
    # more than the fixed 8 Mi
    n, p = 128, 65536
    U = np.linalg.qr(np.random.default_rng(4).standard_normal((n, 128)))[0]
    dbig = c.import_tsvd(U, np.ones(128), U)
    Bbig = torch.zeros((n, p), device="cuda")
    obig = torch.empty((n, p), device="cuda")
    with pytest.raises(AmmError, match="AMM_EUNSUPPORTED"):
        c.approx_matmul_static(dbig, Bbig, obig)

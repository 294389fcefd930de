"""The n = 256 workload: A, B = Q1 diag(exp(-i/20)) Q2^T + 1e-3 N(0, 1) (Haar
Q, seeded).  Circulant K = 16 made on the device and truncated SVD k = 16
(the oracle's exact factors imported, and the device's randomized SVD), zeroth
and first order (Alg. 2.3, eq. (2.1)), each against the float64 oracle on the
same decomposition and against the exact product AB."""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import product as op
from oracle import tsvd as ot
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel

pytestmark = pytest.mark.gpu

N, K = 256, 16


@pytest.fixture(scope="module")
def pair():
    p = inputs.workload_exp_decay(N)
    return f32(p.A), f32(p.B)


@pytest.mark.parametrize("order", ["zeroth", "first"])
def test_circulant_k16(pair, order):
    A, B = pair
    note(f"exp-decay n={N} circulant K={K} {order}")
    c = ctx()
    dA, dB = c.decompose(gpu(A), "circulant", K), c.decompose(gpu(B), "circulant", K)
    oA, oB = oc.CirculantDecomp(A, K), oc.CirculantDecomp(B, K)
    assert list(dA.frequencies()) == list(oA.S) and list(dB.frequencies()) == list(oB.S)
    second = dB if order == "first" else None
    got = host(c.approx_matmul(dA, gpu(B), second))
    want = np.real(op.algorithm(oA, B, oB if order == "first" else None))
    assert rel(got, want) < TOL_F32
    exact = A @ B
    e_gpu, e_or = rel(got, exact), rel(want, exact)
    note(f"  err vs AB {e_gpu:.4e} (oracle {e_or:.4e})")
    assert abs(e_gpu - e_or) <= 1e-5 * max(e_or, 1.0)


@pytest.mark.parametrize("order", ["zeroth", "first"])
def test_tsvd_k16(pair, order):
    A, B = pair
    note(f"exp-decay n={N} tsvd k={K} {order}")
    c = ctx()
    tA, tB = ot.TSVDDecomp(A, K), ot.TSVDDecomp(B, K)
    sA = c.import_tsvd(tA.U, tA.s, tA.V, A=gpu(A))
    sB = c.import_tsvd(tB.U, tB.s, tB.V)
    got = host(c.approx_matmul(sA, gpu(B), sB if order == "first" else None))
    want = op.algorithm(tA, B, tB if order == "first" else None)
    assert rel(got, want) < TOL_F32
    # the device's randomized SVD at the same rank: within 1 % of the exact
    # truncation's error against AB (sigma falls by exp(-1/20) per index, so
    # the sketch with oversampling and power iterations resolves it)
    exact = A @ B
    rA, rB = c.decompose(gpu(A), "tsvd", K, seed=5), c.decompose(gpu(B), "tsvd", K, seed=6)
    got_r = host(c.approx_matmul(rA, gpu(B), rB if order == "first" else None))
    e_r, e_x = rel(got_r, exact), rel(want, exact)
    note(f"  err vs AB: rSVD {e_r:.4e}, exact SVD {e_x:.4e}")
    assert e_r <= 1.01 * e_x + 1e-6

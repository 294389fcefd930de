"""First-order products with different decompositions for A and B (eq. (2.1)
needs only A = Atil + Delta A and B = Btil + Delta B): every pairing of
circulant, truncated SVD and dominant-entry splits, through the C ABI, against
the float64 oracle on identical decompositions."""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import product as op
from oracle import sparse as osp
from oracle import tsvd as ot
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel

pytestmark = pytest.mark.gpu

FRAC = 0.02


def _operand(n, seed):
    """Low-rank decay plus a Toeplitz part plus a few large entries: every
    decomposition has something to keep."""
    rng = np.random.default_rng(seed)
    A = inputs.spectral_matrix(n, n, inputs.decay_power(n, 1.2), rng)
    A = A + 0.02 * inputs.toeplitz_uniform(n, rng)
    pos, vals = inputs.sparse_overlay(n, n, FRAC, 0.5, rng)
    A.reshape(-1)[pos] += vals
    return f32(A)


def _build(c, kind, M, K):
    """(oracle decomposition, device handle) of the same decomposition."""
    Mg = gpu(M)
    if kind == "circulant":
        dec = oc.CirculantDecomp(M, K)
        d = c.decompose(Mg, "circulant", K)
        assert list(d.frequencies()) == list(dec.S)
    elif kind == "tsvd":
        dec = ot.TSVDDecomp(M, K)
        d = c.import_tsvd(dec.U, dec.s, dec.V, A=Mg)
    elif kind == "sparse-tsvd":
        dec = osp.SparseDecomp(M, FRAC, "tsvd", K)
        res = c.import_tsvd(dec.inner.U, dec.inner.s, dec.inner.V, A=gpu(dec.R))
        d = c.import_sparse(M.shape[0], M.shape[1], dec.S.row_ptr, dec.S.col, dec.S.val, residue=res)
    elif kind == "sparse-circ":
        dec = osp.SparseDecomp(M, FRAC, "circulant", K)
        d = c.decompose(Mg, "sparse+circulant", K, sparse_frac=FRAC)
        assert list(d.frequencies()) == list(dec.inner.S)
    else:
        dec = osp.SparseDecomp(M, FRAC)
        d = c.decompose(Mg, "sparse", 0, sparse_frac=FRAC)
    return dec, d, Mg


PAIRS = [("circulant", "tsvd"), ("tsvd", "circulant"), ("sparse-tsvd", "circulant"), ("circulant", "sparse-tsvd"),
         ("sparse", "tsvd"), ("tsvd", "sparse-circ"), ("sparse-circ", "sparse"), ("sparse-tsvd", "sparse-circ")]


@pytest.mark.parametrize("ka,kb", PAIRS)
def test_mixed_first_order_parity(ka, kb):
    n = 256
    note(f"mixed first order {ka} x {kb}")
    A, B = _operand(n, 3), _operand(n, 4)
    c = ctx()
    decA, dA, Ag = _build(c, ka, A, 6)
    decB, dB, Bg = _build(c, kb, B, 8)
    got = host(c.approx_matmul(dA, Bg, dB))
    want = op.algorithm(decA, B, decB)
    assert rel(got, want) < TOL_F32
    # the norm-based estimates apply to any pairing whose handles know their norms
    # (an imported sparse split does not)
    est = c.estimate_error(dA, dB, gpu(got))
    known = "sparse-tsvd" not in (ka, kb)
    assert np.isfinite(est["posterior"]) == known
    if known:
        nA, nB = np.linalg.norm(A), np.linalg.norm(B)
        ndA = np.linalg.norm(np.real(decA.residual_dense()))
        ndB = np.linalg.norm(np.real(decB.residual_dense()))
        assert abs(est["prior"] - ndA * ndB / (nA * nB)) <= 2e-4 * est["prior"]


def test_mixed_first_order_identity_at_1024():
    """M1 = AB - Delta A Delta B for circulant A and truncated-SVD B at n = 1024."""
    n = 1024
    A, B = _operand(n, 13), _operand(n, 14)
    c = ctx()
    decA, dA, Ag = _build(c, "circulant", A, 16)
    decB, dB, Bg = _build(c, "tsvd", B, 24)
    got = host(c.approx_matmul(dA, Bg, dB))
    dAm = A - np.real(decA.truncated_dense())
    dBm = B - decB.truncated_dense()
    assert rel(got, A @ B - dAm @ dBm) < TOL_F32

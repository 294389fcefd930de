"""The n = 16384 workload (0.5 % Laplace(0, 20) entries over a rank-1024
residue with sigma_i = i^-1.5), decomposed on the device as S + circulant_64(R)
(eq. (2.4) with a truncated residue), checked against the float64 oracle.

The sparse part is checked against the definition of the global top-nnz
selection (as read here: the round(f m n) entries of largest
|a|, ties to the smaller row-major index) without sorting 2^28 entries on the
host: the stored values are A's entries at the stored positions, their count
is round(f m n), every kept |a| is >= every dropped |a|, and at the threshold
value the kept positions precede the dropped ones.  The residue R = A - S is
then decomposed by the oracle (Alg. 2.2/2.3): the kept frequencies must equal
the device's, the eigenvalue lists must agree to float32 rounding, and the
product (float32 and float16 spectral products) must match the oracle's
S B + Atil_R B on sampled output columns."""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import sparse as osp
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu

U16 = 2.0 ** -11


class _Lists:
    def __init__(self, n, S, L):
        self.n, self.S, self.L = n, np.asarray(S, dtype=np.int64), np.asarray(L)


def test_sparse_circulant_n16384_against_oracle():
    torch = torch_cuda()
    n, K, frac = 16384, 64, 0.005
    note(f"sparse + circulant decomposition n={n} K={K} frac={frac}")
    pair = inputs.workload_lowrank_sparse(n, device="cuda")
    A = pair.A.float().contiguous()
    B = pair.B.float().contiguous()
    del pair
    torch.cuda.empty_cache()
    c = ctx()
    d = c.decompose(A, "sparse+circulant", K, sparse_frac=frac)
    nnz = osp.dominant_count(n, n, frac)
    rp, col, val = d.sparse_part()
    assert rp[-1] == nnz and d.info()["nnz"] == nnz
    Ah = host(A)
    rows = np.repeat(np.arange(n), np.diff(rp))
    flat = rows.astype(np.int64) * n + col
    assert np.all(np.diff(rp) >= 0) and np.all(np.diff(flat) > 0)      # row-major order, distinct
    assert np.array_equal(val.astype(np.float64), Ah[rows, col])
    mask = np.zeros(n * n, dtype=bool)
    mask[flat] = True
    absA = np.abs(Ah).reshape(-1)
    kept_min = absA[mask].min()
    dropped = absA[~mask]
    assert kept_min >= dropped.max()
    tie_kept = np.flatnonzero(mask & (absA == kept_min))
    tie_dropped = np.flatnonzero(~mask & (absA == kept_min))
    assert tie_dropped.size == 0 or tie_kept.max() < tie_dropped.min()
    del mask, absA, dropped
    S = osp.CSR(n, n, rp, col, val)
    Rh = Ah.copy()
    Rh[rows, col] = 0.0
    del Ah
    note("  oracle circulant decomposition of the residue")
    dec = oc.CirculantDecomp(Rh, K)
    del Rh
    dec.A = None
    assert list(d.frequencies()) == list(dec.S)
    L = d.lists()
    tol = 2.0 ** -24 * np.abs(dec.L) + 1e-12 * np.max(np.abs(dec.L))
    assert np.all(np.abs(L.real - dec.L.real) <= tol) and np.all(np.abs(L.imag - dec.L.imag) <= tol)
    cols = np.sort(np.random.default_rng(55).choice(n, 32, replace=False))
    Bc = host(B[:, torch.from_numpy(cols).cuda()])
    sb = osp.spmm(S, Bc)
    cd = np.real(oc.apply_zeroth(dec, Bc))
    want = sb + cd
    got = host(c.approx_matmul(d, B)[:, torch.from_numpy(cols).cuda()])
    err = rel(got, want)
    note(f"  float32 spectral products: err vs oracle {err:.2e}")
    assert err < TOL_F32
    d.set_spectral_fp16(True)
    got16 = host(c.approx_matmul(d, B)[:, torch.from_numpy(cols).cuda()])
    terms = sum(np.linalg.norm(np.real(oc.apply_zeroth(_Lists(n, [k], dec.L[t:t + 1]), Bc)))
                for t, k in enumerate(dec.S))
    bound = 2.0 * U16 * (1.0 + U16) * terms / np.linalg.norm(want) + TOL_F32
    err16 = rel(got16, want)
    note(f"  float16 spectral products: err vs oracle {err16:.2e} (bound {bound:.2e}); circulant term "
         f"{np.linalg.norm(cd) / np.linalg.norm(want):.2e} of the product")
    assert err16 < bound

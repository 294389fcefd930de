"""GPU parity of the circulant path against the float64 oracle (through the C ABI).

Products are checked on identical decompositions (the oracle's frequency set
and eigenvalue lists imported into the library) to the float32 bar 1e-5
relative Frobenius; the device decomposition is checked on its energies
(float64), its frequency set (exact), and on the product it yields.
"""
import numpy as np
import pytest

from oracle import circulant as oc
from oracle import product as op
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu


def _import(c, dec, residual=None):
    return c.import_circulant(dec.n, dec.S, dec.L, residual=residual)


@pytest.mark.parametrize("n,p,K", [
    (2, 3, 1), (4, 5, 2), (8, 1, 3), (16, 33, 5), (32, 64, 7), (64, 70, 10),
    (128, 31, 20), (256, 256, 16), (512, 100, 33), (1024, 50, 64), (2048, 40, 16),
    (4096, 24, 8),
])
def test_apply_parity_small(n, p, K):
    note(f"cd apply parity n={n} p={p} K={K}")
    rng = np.random.default_rng(1000 + n + p)
    A = f32(rng.standard_normal((n, n)))
    B = f32(rng.standard_normal((n, p)))
    dec = oc.CirculantDecomp(A, K)
    want = np.real(oc.apply_zeroth(dec, B))
    c = ctx()
    d = _import(c, dec)
    got = host(c.approx_matmul(d, gpu(B)))
    assert got.shape == (n, p)
    assert rel(got, want) < TOL_F32


def test_apply_zero_components_and_empty():
    c = ctx()
    n = 64
    B = f32(np.random.default_rng(3).standard_normal((n, 10)))
    d = c.import_circulant(n, [], np.zeros((0, n)))
    out = gpu(np.full((n, 10), 7.0))
    got = host(c.approx_matmul(d, gpu(B), out=out))
    assert np.all(got == 0)


@pytest.mark.parametrize("K", [8, 32, 128])
def test_apply_full_size_sampled(K):
    """n = 4096 square product over all 4096 columns in the launch the bench
    times; the oracle checks 48 sampled columns one by one."""
    torch = torch_cuda()
    n = 4096
    note(f"cd apply full size n={n} K={K}")
    pair = inputs.workload_power_decay(n, device="cuda")
    A = pair.A.float()
    B = pair.B.float()
    Ah = A.double().cpu().numpy()
    dec = oc.CirculantDecomp(Ah, K)
    c = ctx()
    d = _import(c, dec)
    out = c.approx_matmul(d, B)
    torch.cuda.synchronize()
    cols = np.sort(np.random.default_rng(K).choice(n, 48, replace=False))
    Bs = B[:, cols].double().cpu().numpy()
    want = np.real(oc.apply_zeroth(dec, Bs))
    got = out[:, cols].double().cpu().numpy()
    assert rel(got, want) < TOL_F32


@pytest.mark.parametrize("n,KA,KB", [(16, 3, 5), (64, 9, 4), (256, 16, 16), (1024, 33, 8)])
def test_first_order_parity(n, KA, KB):
    note(f"cd first order n={n} KA={KA} KB={KB}")
    rng = np.random.default_rng(n + KA)
    A = f32(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    B = f32(inputs.toeplitz_uniform(n, rng) + 0.1 * rng.standard_normal((n, n)))
    decA = oc.CirculantDecomp(A, KA)
    decB = oc.CirculantDecomp(B, KB)
    want = op.algorithm(decA, B, decB)
    c = ctx()
    res = gpu(np.real(decA.residual_dense()))
    dA = _import(c, decA, residual=res)
    dB = _import(c, decB)
    got = host(c.approx_matmul(dA, gpu(B), dB))
    assert rel(got, want) < TOL_F32


def _selection_is_stable(E, K):
    """The selection does not move under 1e-9 relative perturbations of E, so
    device and host energies (equal to ~1e-15) must pick the same set."""
    base = list(oc.select_pair_closed(E, K))
    rng = np.random.default_rng(0)
    for _ in range(8):
        Ep = E * (1 + 1e-9 * rng.uniform(-1, 1, size=E.shape))
        if list(oc.select_pair_closed(Ep, K)) != base:
            return False
    return True


@pytest.mark.parametrize("n,K", [(2, 1), (4, 2), (16, 5), (64, 8), (256, 16), (1024, 40)])
def test_decompose_parity(n, K):
    note(f"cd decompose n={n} K={K}")
    rng = np.random.default_rng(7 * n + K)
    A = f32(inputs.toeplitz_uniform(n, rng) + 0.05 * rng.standard_normal((n, n)))
    B = f32(rng.standard_normal((n, 12)))
    dec = oc.CirculantDecomp(A, K)
    c = ctx()
    Ag = gpu(A)
    d = c.decompose(Ag, "circulant", K)
    E = d.energies()
    assert np.max(np.abs(E - dec.E)) <= 1e-11 * np.max(dec.E)
    S = d.frequencies()
    assert _selection_is_stable(dec.E, K)
    assert list(S) == list(dec.S)
    inf = d.info()
    assert inf["K_eff"] == len(dec.S)
    assert np.isclose(inf["norm_residual"], dec.norm_residual(), rtol=1e-9, atol=1e-12)
    # eigenvalue lists (Alg. 2.3 step 4) directly: float64 on the device, kept
    # as float32, so each part within its float32 rounding of the oracle's value
    L = d.lists()
    assert L.shape == dec.L.shape
    tol = 2.0 ** -24 * np.abs(dec.L) + 1e-12 * np.max(np.abs(dec.L))
    assert np.all(np.abs(L.real - dec.L.real) <= tol) and np.all(np.abs(L.imag - dec.L.imag) <= tol)
    got = host(c.approx_matmul(d, gpu(B)))
    assert rel(got, np.real(oc.apply_zeroth(dec, B))) < TOL_F32


@pytest.mark.parametrize("n,K", [(64, 4), (512, 6)])
def test_decompose_first_order_residual(n, K):
    """Delta A kept by the device decomposition drives the first-order term."""
    rng = np.random.default_rng(n)
    A = f32(inputs.toeplitz_uniform(n, rng))
    B = f32(inputs.toeplitz_uniform(n, rng))
    decA, decB = oc.CirculantDecomp(A, K), oc.CirculantDecomp(B, K)
    want = op.algorithm(decA, B, decB)
    c = ctx()
    dA = c.decompose(gpu(A), "circulant", K)
    dB = c.decompose(gpu(B), "circulant", K)
    got = host(c.approx_matmul(dA, gpu(B), dB))
    assert rel(got, want) < TOL_F32


def test_planted_modes_recovered():
    """A planted set of classes is found exactly and reproduced."""
    n = 256
    rng = np.random.default_rng(5)
    A = f32(inputs.planted_circulant(n, [0, 3, 17, 100], rng, noise=1e-3))
    c = ctx()
    d = c.decompose(gpu(A), "circulant", 7)
    assert sorted(d.frequencies()) == sorted([0, 3, n - 3, 17, n - 17, 100, n - 100])


def test_rejects_unsupported():
    from paper_2504_19308_amd import AmmError
    c = ctx()
    with pytest.raises(AmmError):   # side 1 (any side in [2, 16384] is supported)
        c.decompose(gpu(np.zeros((1, 1))), "circulant", 1)
    with pytest.raises(AmmError):   # rectangular: blocks of side min(m, n) = 1
        c.decompose(gpu(np.zeros((8, 1))), "circulant", 1)
    with pytest.raises(AmmError):   # more components than the side
        c.decompose(gpu(np.zeros((6, 6))), "circulant", 7)

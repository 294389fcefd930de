"""Batched truncated-SVD products (many uneven (A, B) pairs, two launches,
graph replay) against the float64 oracle, entry by entry."""
import numpy as np
import pytest

from oracle import tsvd as ot
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, bf16, ctx, f32, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu

SHAPES = [(256, 256), (512, 256), (256, 512), (384, 128), (128, 640)]


def _batch(c, k, p, count, seed=0):
    rng = np.random.default_rng(seed)
    decs, Bs, wants, keep = [], [], [], []
    for i in range(count):
        m, n = SHAPES[i % len(SHAPES)]
        A = f32(inputs.spectral_matrix(m, n, inputs.decay_power(min(m, n), 1.0), rng))
        B = f32(rng.standard_normal((n, p)))
        dec = ot.TSVDDecomp(A, k)
        decs.append(c.import_tsvd(dec.U, dec.s, dec.V))
        Bs.append(gpu(B))
        wants.append(ot.apply_zeroth(dec, B))
    return decs, Bs, wants


@pytest.mark.parametrize("k,p,count", [(32, 256, 7), (128, 128, 5), (16, 384, 12)])
def test_batch_matches_oracle(k, p, count):
    note(f"batch k={k} p={p} count={count}")
    c = ctx()
    decs, Bs, wants = _batch(c, k, p, count, seed=k + count)
    plan = c.batch_plan(decs, Bs)
    outs = plan.run(use_graph=False)
    for o, w in zip(outs, wants):
        assert rel(host(o), w) < TOL_F32
    info = plan.info()
    assert info["panel_blocks"] > 0 and info["out_blocks"] > 0


def test_batch_graph_replays_match_eager():
    torch = torch_cuda()
    c = ctx()
    decs, Bs, wants = _batch(c, 32, 256, 6, seed=9)
    plan = c.batch_plan(decs, Bs)
    eager = [o.clone() for o in plan.run(use_graph=False)]
    torch.cuda.synchronize()
    for rep in range(4):
        for o in plan.outs:
            o.fill_(float("nan"))          # eager work between replays
        torch.cuda.synchronize()
        plan.run(use_graph=True)
        torch.cuda.synchronize()
        for o, e in zip(plan.outs, eager):
            assert torch.equal(o, e), f"replay {rep} differs"
    for o, w in zip(eager, wants):
        assert rel(host(o), w) < TOL_F32


def test_batch_rejects_mixed_ranks():
    from paper_2504_19308_amd import AmmError
    c = ctx()
    d1, B1, _ = _batch(c, 32, 128, 1, seed=1)
    d2, B2, _ = _batch(c, 16, 128, 1, seed=2)
    with pytest.raises(AmmError):
        c.batch_plan(d1 + d2, B1 + B2)


class _Factors:
    """Given truncated-SVD factors (what the oracle's product reads)."""

    def __init__(self, U, s, V):
        self.U, self.s, self.V = U, s, V


def test_batch_full_size_sampled():
    """The 64-pair uneven batch at full size (4096 x 4096, 11008 x 4096,
    4096 x 11008 by pair index mod 3; rank 128; 2048 columns), replayed as a
    graph like the benchmark; every pair checked on sampled output columns."""
    torch = torch_cuda()
    note("batch full size 64 pairs")
    shapes = [(4096, 4096), (11008, 4096), (4096, 11008)]
    k, p, count = 128, 2048, 64
    c = ctx()
    g = torch.Generator(device="cuda")
    g.manual_seed(inputs.seed_of(3, 1))
    decs, Bs, facs = [], [], []
    for i in range(count):
        m, n = shapes[i % 3]
        rng = inputs.rng_of(3, 0, i)
        sig = inputs.decay_power(min(m, n), 1.0)[:k]
        U = inputs.haar_columns(m, k, rng, device="cuda").cpu().numpy()
        V = inputs.haar_columns(n, k, rng, device="cuda").cpu().numpy()
        decs.append(c.import_tsvd(U, sig, V))
        # the factors the library holds are float32: the oracle uses the same
        facs.append(_Factors(f32(U), f32(sig), f32(V)))
        Bs.append(torch.randn((n, p), generator=g, device="cuda", dtype=torch.float32))
    plan = c.batch_plan(decs, Bs)
    plan.run(use_graph=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(64)
    for i in range(count):
        cols = np.sort(rng.choice(p, 6, replace=False))
        want = ot.apply_zeroth(facs[i], Bs[i][:, cols].double().cpu().numpy())
        got = plan.outs[i][:, cols].double().cpu().numpy()
        assert rel(got, want) < TOL_F32, f"pair {i}"


def _batch_bf16(c, k, p, count, seed=0):
    """Pairs whose B_i are bfloat16; the oracle multiplies the bfloat16
    components the plan holds: bf16(float32(U S)), bf16(float32(V)), bf16(B)."""
    torch = torch_cuda()
    rng = np.random.default_rng(seed)
    decs, Bs, wants = [], [], []
    for i in range(count):
        m, n = SHAPES[i % len(SHAPES)]
        A = f32(inputs.spectral_matrix(m, n, inputs.decay_power(min(m, n), 1.0), rng))
        dec = ot.TSVDDecomp(A, k)
        decs.append(c.import_tsvd(dec.U, dec.s, dec.V))
        B = rng.standard_normal((n, p)).astype(np.float32)
        Bs.append(torch.from_numpy(B).cuda().bfloat16())
        US = bf16((dec.U * dec.s[None, :]).astype(np.float32))
        V = bf16(dec.V.astype(np.float32))
        wants.append(ot.apply_zeroth(_Factors(US, np.ones(k), V), bf16(B)))
    return decs, Bs, wants


@pytest.mark.parametrize("k,p,count", [(32, 256, 7), (128, 128, 5), (64, 384, 6)])
def test_batch_bf16_matches_oracle(k, p, count):
    note(f"batch bf16 k={k} p={p} count={count}")
    c = ctx()
    decs, Bs, wants = _batch_bf16(c, k, p, count, seed=3 * k + count)
    plan = c.batch_plan(decs, Bs)
    outs = plan.run(use_graph=False)
    for o, w in zip(outs, wants):
        assert rel(host(o), w) < TOL_F32


def test_batch_bf16_graph_replays_match_eager():
    torch = torch_cuda()
    c = ctx()
    decs, Bs, wants = _batch_bf16(c, 64, 256, 5, seed=11)
    plan = c.batch_plan(decs, Bs)
    eager = [o.clone() for o in plan.run(use_graph=False)]
    torch.cuda.synchronize()
    for rep in range(3):
        for o in plan.outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.run(use_graph=True)
        torch.cuda.synchronize()
        for o, e in zip(plan.outs, eager):
            assert torch.equal(o, e), f"replay {rep} differs"
    for o, w in zip(eager, wants):
        assert rel(host(o), w) < TOL_F32


def test_batch_bf16_rejects_unaligned():
    from paper_2504_19308_amd import AmmError
    torch = torch_cuda()
    c = ctx()
    rng = np.random.default_rng(0)
    A = f32(inputs.spectral_matrix(128, 100, inputs.decay_power(100, 1.0), rng))   # n = 100: not a multiple of 32
    dec = ot.TSVDDecomp(A, 32)
    d = c.import_tsvd(dec.U, dec.s, dec.V)
    with pytest.raises(AmmError):
        c.batch_plan([d], [torch.zeros((100, 128), device="cuda", dtype=torch.bfloat16)])


def test_batch_bf16_full_size_sampled():
    """The 64-pair uneven batch at full size with bfloat16 activations and
    components, graph replay, every pair checked on sampled columns."""
    torch = torch_cuda()
    note("batch bf16 full size 64 pairs")
    shapes = [(4096, 4096), (11008, 4096), (4096, 11008)]
    k, p, count = 128, 2048, 64
    c = ctx()
    g = torch.Generator(device="cuda")
    g.manual_seed(inputs.seed_of(3, 2))
    decs, Bs, facs = [], [], []
    for i in range(count):
        m, n = shapes[i % 3]
        rng = inputs.rng_of(3, 0, i)
        sig = inputs.decay_power(min(m, n), 1.0)[:k]
        U = inputs.haar_columns(m, k, rng, device="cuda").cpu().numpy()
        V = inputs.haar_columns(n, k, rng, device="cuda").cpu().numpy()
        decs.append(c.import_tsvd(U, sig, V))
        facs.append(_Factors(bf16((U * sig[None, :]).astype(np.float32)), np.ones(k), bf16(V.astype(np.float32))))
        Bs.append(torch.randn((n, p), generator=g, device="cuda", dtype=torch.float32).bfloat16())
    plan = c.batch_plan(decs, Bs)
    plan.run(use_graph=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(65)
    for i in range(count):
        cols = np.sort(rng.choice(p, 6, replace=False))
        want = ot.apply_zeroth(facs[i], Bs[i][:, cols].double().cpu().numpy())
        got = plan.outs[i][:, cols].double().cpu().numpy()
        assert rel(got, want) < TOL_F32, f"pair {i}"

"""Rectangular operands as square circulant blocks (Sec. 2.3; the last block
zero-padded) and circulant batch plans, against the float64 oracle."""
import numpy as np
import pytest

from oracle import circulant as oc
from paper_2504_19308_amd import inputs
from tests._gpu_common import TOL_F32, ctx, f32, gpu, host, note, rel, torch_cuda

pytestmark = pytest.mark.gpu


def _rect_toeplitz(m, n, seed):
    """A rectangular slice of a U(0,1) Toeplitz matrix plus a little noise:
    strong, well separated circulant components in every block."""
    rng = np.random.default_rng(seed)
    T = inputs.toeplitz_uniform(max(m, n), rng)[:m, :n]
    return f32(T + 0.05 * rng.standard_normal((m, n)))


def _stable(E, K):
    base = list(oc.select_pair_closed(E, K))
    rng = np.random.default_rng(0)
    return all(list(oc.select_pair_closed(E * (1 + 1e-9 * rng.uniform(-1, 1, E.shape)), K)) == base
               for _ in range(8))


@pytest.mark.parametrize("m,n,K", [(200, 64, 5), (64, 150, 4), (256, 512, 9), (1000, 128, 3), (128, 128, 6)])
def test_blocked_decompose_and_apply(m, n, K):
    note(f"blocked circulant m={m} n={n} K={K}")
    A = _rect_toeplitz(m, n, m + n + K)
    B = f32(np.random.default_rng(K).standard_normal((n, 33)))
    dec = oc.BlockedCirculant(A, K)
    c = ctx()
    d = c.decompose(gpu(A), "circulant", K)
    inf = d.info()
    assert inf["blocks"] == (dec.nb if m != n else 0)
    if m != n:
        for j, blk in enumerate(dec.blocks):
            assert _stable(blk.E, K)
            b = d.block(j)
            assert list(b.frequencies()) == list(blk.S)
            assert np.max(np.abs(b.energies() - blk.E)) <= 1e-11 * np.max(blk.E)
    got = host(c.approx_matmul(d, gpu(B)))
    assert rel(got, oc.apply_blocked(dec, B)) < TOL_F32


def test_blocked_first_order_is_rejected():
    from paper_2504_19308_amd import AmmError
    A = _rect_toeplitz(128, 64, 1)
    c = ctx()
    d = c.decompose(gpu(A), "circulant", 3)
    B = f32(np.random.default_rng(2).standard_normal((64, 64)))
    dB = c.decompose(gpu(B), "circulant", 3)
    with pytest.raises(AmmError):
        c.approx_matmul(d, gpu(B), dB)


def test_blocked_full_expansion_at_full_size():
    """11008 x 4096 and 4096 x 11008 with every component of every block
    (K = 4096): the blocked product is A B exactly (checked on sampled columns
    against a float64 product)."""
    torch = torch_cuda()
    c = ctx()
    g = torch.Generator(device="cuda")
    g.manual_seed(inputs.seed_of(3, 7))
    for (m, n) in ((11008, 4096), (4096, 11008)):
        note(f"blocked full expansion {m}x{n}")
        A = torch.randn((m, n), generator=g, device="cuda", dtype=torch.float32)
        B = torch.randn((n, 256), generator=g, device="cuda", dtype=torch.float32)
        d = c.decompose(A, "circulant", 4096)
        assert d.info()["blocks"] == 3
        out = c.approx_matmul(d, B)
        cols = torch.arange(0, 256, 16, device="cuda")
        want = A.double() @ B[:, cols].double()
        got = out[:, cols].double()
        assert float((got - want).norm() / want.norm()) < TOL_F32
        del A, B, out, d
        torch.cuda.empty_cache()


def test_circulant_batch_plan():
    """Square and blocked circulant entries of different sizes in one plan,
    graph replays identical to the eager run and to the oracle."""
    torch = torch_cuda()
    c = ctx()
    shapes = [(64, 64, 5, 40), (200, 64, 4, 33), (64, 150, 3, 17), (256, 256, 8, 128), (128, 512, 6, 64)]
    decs, Bs, wants = [], [], []
    for i, (m, n, K, p) in enumerate(shapes):
        A = _rect_toeplitz(m, n, 50 + i)
        B = f32(np.random.default_rng(60 + i).standard_normal((n, p)))
        decs.append(c.decompose(gpu(A), "circulant", K))
        Bs.append(gpu(B))
        if m == n:
            wants.append(np.real(oc.apply_zeroth(oc.CirculantDecomp(A, K), B)))
        else:
            wants.append(oc.apply_blocked(oc.BlockedCirculant(A, K), B))
    plan = c.batch_plan(decs, Bs)
    eager = [o.clone() for o in plan.run(use_graph=False)]
    torch.cuda.synchronize()
    for o, w in zip(eager, wants):
        assert rel(host(o), w) < TOL_F32
    for rep in range(3):
        for o in plan.outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.run(use_graph=True)
        torch.cuda.synchronize()
        for o, e in zip(plan.outs, eager):
            assert torch.equal(o, e), f"replay {rep} differs"


def test_mixed_batch_is_rejected():
    from paper_2504_19308_amd import AmmError
    from oracle import tsvd as ot
    torch = torch_cuda()
    c = ctx()
    A = _rect_toeplitz(128, 128, 9)
    dc = c.decompose(gpu(A), "circulant", 4)
    dec = ot.TSVDDecomp(A, 16)
    dt = c.import_tsvd(dec.U, dec.s, dec.V)
    B = gpu(np.ones((128, 128)))
    with pytest.raises(AmmError):
        c.batch_plan([dc, dt], [B, B])


def test_circulant_batch_job_table_matches_entry_launches():
    """The batched job-table launches against the per-entry launches, bit for
    bit, on square, row-blocked and column-blocked entries (partial last
    blocks, odd column counts, a zero-rank entry, float16 lists) next to a
    side that only runs per entry; graph replays of the job table; and the
    tuner's report."""
    torch = torch_cuda()
    c = ctx()
    shapes = [(64, 64, 5, 40), (200, 64, 4, 33), (64, 150, 3, 17), (256, 256, 8, 128), (128, 512, 6, 64),
              (1024, 1024, 0, 24), (2500, 1024, 6, 24), (1024, 2500, 6, 20), (300, 300, 5, 20)]
    decs, Bs = [], []
    for i, (m, n, K, p) in enumerate(shapes):
        A = _rect_toeplitz(m, n, 80 + i)
        decs.append(c.decompose(gpu(A), "circulant", K))
        Bs.append(gpu(np.random.default_rng(90 + i).standard_normal((n, p))))
    A = _rect_toeplitz(1024, 1024, 99)
    decs.append(c.decompose(gpu(A), "circulant", 12, spectral_fp16=True))
    Bs.append(gpu(np.random.default_rng(98).standard_normal((1024, 48))))
    plan = c.batch_plan(decs, Bs)
    sched = plan.circulant_schedule()
    note(f"  schedule {sched}")
    assert sched["entry_ms"] > 0 and sched["table_ms"] > 0
    results = {}
    for mode in (False, True):
        plan.set_circulant_mode(mode)
        assert plan.circulant_schedule()["job_table"] == mode
        for o in plan.outs:
            o.fill_(float("nan"))
        results[mode] = [o.clone() for o in plan.run(use_graph=False)]
        torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(results[False], results[True])):
        assert torch.equal(a, b), f"entry {i} differs between the schedules"
    assert float(results[True][5].abs().max()) == 0.0          # zero rank: zero product
    for i in (0, 3):                                            # square entries against the oracle
        m, n, K, p = shapes[i]
        Ah = _rect_toeplitz(m, n, 80 + i)
        want = np.real(oc.apply_zeroth(oc.CirculantDecomp(Ah, K), host(Bs[i])))
        assert rel(host(results[True][i]), want) < TOL_F32
    for rep in range(3):
        for o in plan.outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.run(use_graph=True)
        torch.cuda.synchronize()
        for o, e in zip(plan.outs, results[True]):
            assert torch.equal(o, e), f"replay {rep} differs"


def test_circulant_batch_bf16():
    """bfloat16 B_i through the job table: equal to the float32 plan on the
    widened values; sides the batched launches do not cover are refused."""
    from paper_2504_19308_amd import AmmError
    torch = torch_cuda()
    c = ctx()
    shapes = [(256, 256, 8, 64), (600, 256, 5, 36), (256, 700, 4, 40), (1024, 1024, 10, 96)]
    decs, B16 = [], []
    for i, (m, n, K, p) in enumerate(shapes):
        A = _rect_toeplitz(m, n, 70 + i)
        decs.append(c.decompose(gpu(A), "circulant", K, spectral_fp16=(n == 1024)))
        B16.append(gpu(np.random.default_rng(75 + i).standard_normal((n, p))).bfloat16())
    plan16 = c.batch_plan(decs, B16)
    assert plan16.circulant_schedule()["job_table"] and plan16.circulant_schedule()["entry_ms"] < 0
    out16 = [o.clone() for o in plan16.run(use_graph=True)]
    plan32 = c.batch_plan(decs, [b.float() for b in B16]).set_circulant_mode(True)
    out32 = plan32.run(use_graph=False)
    torch.cuda.synchronize()
    for a, b in zip(out16, out32):
        assert torch.equal(a, b)
    odd = c.decompose(gpu(_rect_toeplitz(300, 300, 5)), "circulant", 4)
    with pytest.raises(AmmError):
        c.batch_plan([odd], [gpu(np.ones((300, 8))).bfloat16()])

"""Tune cache (amm_ctx_set_tune_cache): a batch plan's tuned choice is stored
once per device and shapes, and a second plan with the same shapes takes it
from the file without timing; its products equal the tuned plan's."""
import numpy as np
import pytest

from paper_2504_19308_amd import inputs
from tests._gpu_common import ctx, gpu, note, torch_cuda

pytestmark = pytest.mark.gpu


def _tsvd_batch(c, rng):
    from oracle import tsvd as ot
    decs, Bs = [], []
    for i, (m, n, p) in enumerate([(256, 384, 128), (512, 256, 256), (384, 384, 128)]):
        A = rng.standard_normal((m, n)) * np.arange(1, n + 1) ** -1.0
        d = ot.TSVDDecomp(A, 32)
        decs.append(c.import_tsvd(d.U, d.s, d.V))
        Bs.append(gpu(rng.standard_normal((n, p))))
    return decs, Bs


def test_tune_cache_round_trip(tmp_path):
    torch = torch_cuda()
    path = tmp_path / "tune.txt"
    rng = np.random.default_rng(5)
    c = ctx().set_tune_cache(path)
    decs, Bs = _tsvd_batch(c, rng)
    p1 = c.batch_plan(decs, Bs)
    assert not p1.info()["from_cache"]
    out1 = [o.clone() for o in p1.run(use_graph=False)]
    lines = path.read_text().splitlines()
    note(f"  cache: {lines}")
    assert len(lines) == 1 and lines[0].startswith("AMMTUNE1 ")
    p2 = c.batch_plan(decs, Bs)
    info = p2.info()
    assert info["from_cache"] and info["target_blocks"] == p1.info()["target_blocks"]
    out2 = p2.run(use_graph=True)
    torch.cuda.synchronize()
    for a, b in zip(out1, out2):
        assert torch.equal(a, b)
    assert len(path.read_text().splitlines()) == 1          # a hit adds nothing
    # circulant plans: the schedule is cached too; other shapes miss
    n = 1024
    A = gpu(inputs.toeplitz_uniform(n, rng))
    d = c.decompose(A, "circulant", 8)
    Bc = [gpu(rng.standard_normal((n, 32))) for _ in range(2)]
    q1 = c.batch_plan([d, d], Bc)
    q2 = c.batch_plan([d, d], Bc)
    assert not q1.info()["from_cache"] and q2.info()["from_cache"]
    assert q2.circulant_schedule()["job_table"] == q1.circulant_schedule()["job_table"]
    r1, r2 = [o.clone() for o in q1.run(use_graph=False)], q2.run(use_graph=False)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(r1, r2))
    assert len(path.read_text().splitlines()) == 2


def test_tune_cache_bad_file_is_ignored(tmp_path):
    torch = torch_cuda()
    path = tmp_path / "tune.txt"
    path.write_text("garbage line\nAMMTUNE1 zz 1 2 3\n")
    rng = np.random.default_rng(6)
    c = ctx().set_tune_cache(path)
    decs, Bs = _tsvd_batch(c, rng)
    p = c.batch_plan(decs, Bs)
    assert not p.info()["from_cache"]
    p.run(use_graph=True)
    torch.cuda.synchronize()
    # an unwritable location only disables the cache
    c.set_tune_cache(tmp_path / "no_such_dir" / "tune.txt")
    q = c.batch_plan(decs, Bs)
    assert not q.info()["from_cache"]
    c.set_tune_cache(None)

"""GPU parity of the batched path: every job's result in a fused batch (eager and replayed from
a hipGraph) equals its result alone, and sampled rows equal the stored oracle results for the
64-job mixed batch."""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import coracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2012_03771_amd as cs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from goldens import load  # noqa: E402


def _np(t):
    return t.cpu().numpy().view(np.uint32)


def _alone(job, tune=None):
    b, c, ws = cs.sieve(job, tune)
    torch.cuda.synchronize()
    out = _np(b), _np(c)
    del b, c, ws
    return out


SMALL_MIX = [W.Job(61, 6, 1000, 3000, 500, 10**6), W.Job(131, 1, 7, 5000, 900, 2 * 10**6),
             W.Job(11, 2, 9, 25, 40, 700), W.Job(307, 2, 12345, 4000, 2500, 10**7),
             W.Job(13, 6, 1, 50, 20, 300), W.Job(11, 2, 4, 1, 5, 100),          # no rows
             W.Job(401, 210, 99, 30000, 3000, 10**7), W.Job(211, 210, 1, 1000, 4000, 10**6)]


PATHS = [cs.BATCH_PERSISTENT, cs.BATCH_LANES]
PATH_IDS = ["persistent", "lanes"]


@pytest.mark.parametrize("path", PATHS, ids=PATH_IDS)
@pytest.mark.parametrize("mode,scatter", [(cs.LARGE_G, cs.SCATTER_AUTO), (cs.LARGE_THREE_GAP, cs.SCATTER_AUTO),
                                          (cs.LARGE_THREE_GAP, cs.SCATTER_ATOMIC)],
                         ids=["g", "three_gap", "three_gap_atomic"])
def test_small_batch_equals_alone_and_oracle(mode, scatter, path):
    tunes = [cs.Tune(large_mode=mode, scatter=scatter) for _ in SMALL_MIX]
    batch = cs.Batch(SMALL_MIX, tunes, path=path)
    assert batch.path == path
    bm, ct = batch.alloc_outputs()
    batch.run(bm, ct, use_graph=False)
    torch.cuda.synchronize()
    eager = [(_np(b), _np(c)) for b, c in zip(bm, ct)]
    for rep in range(3):
        for t in bm:
            t.fill_(-1)
        for t in ct:
            t.fill_(-1)
        batch.run(bm, ct, use_graph=True)
        torch.cuda.synchronize()
        _alone(W.Job(97, 30, 10**6, 2000, 1200, 10**6))      # unrelated eager work between replays
        for i, job in enumerate(SMALL_MIX):
            assert np.array_equal(_np(bm[i]), eager[i][0]) and np.array_equal(_np(ct[i]), eager[i][1]), (rep, job)
    d = batch.diag()
    assert d.error_flags == 0
    for i, job in enumerate(SMALL_MIX):
        want_b, want_c = coracle.sieve_job(job)
        assert np.array_equal(eager[i][0], want_b) and np.array_equal(eager[i][1], want_c), job
        a_b, a_c = _alone(job, cs.Tune(large_mode=mode))
        assert np.array_equal(eager[i][0], a_b) and np.array_equal(eager[i][1], a_c), job
    batch.close()


@pytest.mark.parametrize("path", PATHS, ids=PATH_IDS)
def test_mixed_64_job_batch_against_oracle_rows(path):
    g = load("batch_rows.npz")
    jobs = W.batch_jobs(64, seed=0)
    tunes = [cs.Tune(large_mode=cs.LARGE_THREE_GAP) for _ in jobs]
    batch = cs.Batch(jobs, tunes, path=path)
    assert batch.path == path
    bm, ct = batch.alloc_outputs()
    for rep in range(2):
        batch.run(bm, ct, use_graph=True)
        torch.cuda.synchronize()
        checked = 0
        for i, job in enumerate(jobs):
            key = f"job{i}_rows"
            if key not in g.files:
                assert batch.layouts[i].n_m == 0
                continue
            assert tuple(int(x) for x in g[f"job{i}_tuple"]) == job.as_tuple()
            rows = g[key]
            b = _np(bm[i])[rows]
            c = _np(ct[i])[rows]
            assert np.array_equal(b, g[f"job{i}_bits"]) and np.array_equal(c, g[f"job{i}_counts"]), (rep, i, job)
            checked += 1
        assert checked >= 60
    assert batch.diag().error_flags == 0
    # a handful of whole jobs: batch == alone
    for i in (0, 7, 33, 63):
        a_b, a_c = _alone(jobs[i], tunes[i])
        assert np.array_equal(_np(bm[i]), a_b) and np.array_equal(_np(ct[i]), a_c), i
    batch.close()


def test_autotuned_batch_equals_alone():
    from paper_2012_03771_amd.autotune import Autotuner
    jobs = [W.Job(307, 2, 12345, 4000, 2500, 10**7), W.Job(401, 210, 99, 30000, 3000, 10**7),
            W.Job(131, 1, 7, 5000, 900, 2 * 10**6)]
    tuner = Autotuner()
    tunes = tuner.tune_all(jobs)
    assert len(tuner.cache) >= 1 and all(len(t) == len(tuner.candidates) for t in tuner.timings.values())
    batch = cs.Batch(jobs, tunes)
    bm, ct = batch.alloc_outputs()
    batch.run(bm, ct, use_graph=True)
    torch.cuda.synchronize()
    for i, job in enumerate(jobs):
        a_b, a_c = _alone(job)                    # default tuning: outputs do not depend on it
        assert np.array_equal(_np(bm[i]), a_b) and np.array_equal(_np(ct[i]), a_c), job
    batch.close()
    # the whole-batch tuning: path, tile rows, then the per-column threshold rule
    tunes2, opts, timings = tuner.tune_batch(jobs, reps=1)
    assert any(t["thr"] == "44 n_x" for t in timings) and any(t["thr"] == "per job" for t in timings)
    b2 = cs.Batch(jobs, tunes2, **opts)
    bm2, ct2 = b2.alloc_outputs()
    b2.run(bm2, ct2, use_graph=True)
    torch.cuda.synchronize()
    for i, job in enumerate(jobs):
        assert torch.equal(bm[i], bm2[i]) and torch.equal(ct[i], ct2[i]), job
    b2.close()


@pytest.mark.parametrize("mode", [cs.LARGE_G, cs.LARGE_THREE_GAP], ids=["g", "three_gap"])
def test_one_call_batch_equals_handle(mode):
    """cs_sieve_batch (caller's workspace and stream, no graph) gives the handle's outputs."""
    jobs = SMALL_MIX + W.batch_jobs(64, seed=0)[:6]
    tunes = [cs.Tune(large_mode=mode) for _ in jobs]
    batch = cs.Batch(jobs, tunes)
    bm, ct = batch.alloc_outputs()
    batch.run(bm, ct, use_graph=True)
    ws = torch.empty((cs.batch_ws_bytes(jobs, tunes),), dtype=torch.uint8, device="cuda")
    bm2, ct2 = batch.alloc_outputs()
    for t in bm2 + ct2:
        t.fill_(-1)
    cs.sieve_batch(jobs, bm2, ct2, ws, tunes)
    torch.cuda.synchronize()
    for i, job in enumerate(jobs):
        assert torch.equal(bm[i], bm2[i]) and torch.equal(ct[i], ct2[i]), job
    batch.close()


def test_persistent_refuses_mixed_enumerations():
    tunes = [cs.Tune(large_mode=cs.LARGE_G), cs.Tune(large_mode=cs.LARGE_THREE_GAP)]
    with pytest.raises(cs.CsError):
        cs.Batch(SMALL_MIX[:2], tunes, path=cs.BATCH_PERSISTENT)
    b = cs.Batch(SMALL_MIX[:2], tunes)
    assert b.path == cs.BATCH_LANES
    b.close()


@pytest.mark.parametrize("order", [cs.ORDER_LARGE_FIRST, cs.ORDER_SMALL_FIRST, cs.ORDER_BY_JOB],
                         ids=["large_first", "small_first", "by_job"])
@pytest.mark.parametrize("ipt", [256, 2048])
def test_persistent_task_shapes_equal_alone(order, ipt):
    """The persistent kernel's queue order and items per task change only the schedule."""
    tunes = [cs.Tune(large_mode=cs.LARGE_THREE_GAP) for _ in SMALL_MIX]
    batch = cs.Batch(SMALL_MIX, tunes, path=cs.BATCH_PERSISTENT, items_per_task=ipt, order=order, blocks_per_cu=2)
    bm, ct = batch.alloc_outputs()
    batch.run(bm, ct, use_graph=True)
    torch.cuda.synchronize()
    for i, job in enumerate(SMALL_MIX):
        a_b, a_c = _alone(job, tunes[i])
        assert np.array_equal(_np(bm[i]), a_b) and np.array_equal(_np(ct[i]), a_c), job
    d = batch.diag()
    assert d.error_flags == 0 and sum(d.dec_primes) == d.large_primes
    batch.close()

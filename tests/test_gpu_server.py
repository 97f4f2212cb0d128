"""GPU tests of the continuous-batching server: results in the mix equal results alone (and the
oracle on small jobs), jobs arriving while others run are admitted and completed, the memory
budget holds, and K mod p tables are reused across jobs."""
import time

import numpy as np
import pytest

import workloads as W
from oracle import coracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2012_03771_amd as cs  # noqa: E402


def _np(t):
    return t.cpu().numpy().view(np.uint32)


def _alone(job, tune):
    b, c, ws = cs.sieve(job, tune)
    torch.cuda.synchronize()
    out = _np(b), _np(c)
    del b, c, ws
    return out


JOBS = [W.Job(61, 6, 1000, 3000, 500, 10**6), W.Job(131, 1, 7, 5000, 900, 2 * 10**6),
        W.Job(11, 2, 9, 25, 40, 700), W.Job(307, 2, 12345, 4000, 2500, 10**7),
        W.Job(401, 210, 99, 30000, 3000, 10**7), W.Job(211, 210, 1, 1000, 4000, 10**6),
        W.Job(401, 210, 5000, 8000, 3000, 5 * 10**6),      # same (P, d) as an earlier job
        W.Job(11, 2, 4, 1, 5, 100),                          # no rows
        W.Job(503, 210, 10**6, 4000, 7000, 3 * 10**7), W.Job(97, 30, 10**6, 20000, 1200, 5 * 10**6)]


@pytest.mark.parametrize("mode,kmod,scatter", [(cs.LARGE_G, cs.KMOD_AUTO, cs.SCATTER_AUTO),
                                               (cs.LARGE_THREE_GAP, cs.KMOD_AUTO, cs.SCATTER_AUTO),
                                               (cs.LARGE_THREE_GAP, cs.KMOD_TABLE, cs.SCATTER_AUTO),
                                               (cs.LARGE_THREE_GAP, cs.KMOD_AUTO, cs.SCATTER_ATOMIC)],
                         ids=["g", "three_gap", "three_gap_table", "three_gap_atomic"])
def test_served_equals_alone(mode, kmod, scatter):
    """Jobs forming K mod p in their large branch (the default), or sharing one table per (P, d);
    large hits through byte counters (the default) or per-hit atomics."""
    tune = cs.Tune(large_mode=mode, kmod=kmod, scatter=scatter)
    srv = cs.Server(budget_bytes=2 << 30, max_limit=10**8, max_active=4, chunks=3, tune=tune)
    tickets = []
    for i, job in enumerate(JOBS):
        tickets.append(srv.submit(job))
        if i % 3 == 2:
            time.sleep(0.02)                 # later jobs arrive while earlier ones run
    for t in tickets:
        info = srv.wait(t, 120.0)
        assert info.state == 2
    for job, t in zip(JOBS, tickets):
        b, c = srv.fetch(t)
        torch.cuda.synchronize()
        a_b, a_c = _alone(job, tune)
        assert np.array_equal(_np(b), a_b) and np.array_equal(_np(c), a_c), job
        if job.limit <= 10**7 and job.m_inc <= 30000:
            w_b, w_c = coracle.sieve_job(job)
            assert np.array_equal(a_b, w_b) and np.array_equal(a_c, w_c), job
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == len(JOBS) and st["failed"] == 0
    if kmod == cs.KMOD_TABLE:
        assert st["kmod_hits"] >= 1                    # (401, 210) twice
    else:
        assert st["kmod_builds"] == 0 and st["kmod_hits"] == 0
    assert st["iterations"] >= 4
    if scatter == cs.SCATTER_ATOMIC:
        assert st["bytes_iterations"] == 0
    else:
        assert st["bytes_iterations"] == st["iterations"]     # every job here admits the counters
    srv.close()


def test_two_lanes_equal_alone():
    """long_ms small enough that the larger jobs run in the second lane, beside the others."""
    tune = cs.Tune(large_mode=cs.LARGE_THREE_GAP)
    srv = cs.Server(budget_bytes=2 << 30, max_limit=10**8, max_active=4, chunks=1, tune=tune, long_ms=0.5)
    tickets = [srv.submit(job) for job in JOBS]
    for t in tickets:
        assert srv.wait(t, 120.0).state == 2
    for job, t in zip(JOBS, tickets):
        b, c = srv.fetch(t)
        torch.cuda.synchronize()
        a_b, a_c = _alone(job, tune)
        assert np.array_equal(_np(b), a_b) and np.array_equal(_np(c), a_c), job
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == len(JOBS) and st["failed"] == 0 and st["active"] == 0 and st["queued"] == 0
    srv.close()
    with pytest.raises(cs.CsError):
        cs.Server(budget_bytes=1 << 20, max_limit=10**6, long_ms=-1.0)


def test_iterations_fall_back_to_atomics_for_a_job_without_byte_counters():
    """A job whose numbers may have 256 or more prime factors above its threshold (2003#, sl = 5:
    threshold 2003) gets no byte counters; the iterations it is in use per-hit atomics for every
    job, and every result still equals the job alone (and the oracle)."""
    odd = W.Job(2003, 1, 1, 50, 5, 10**5)
    assert cs.plan(odd, cs.Tune(large_mode=cs.LARGE_THREE_GAP)).scatter == cs.SCATTER_ATOMIC
    jobs = [JOBS[0], odd, JOBS[3], JOBS[5]]
    tune = cs.Tune(large_mode=cs.LARGE_THREE_GAP)
    srv = cs.Server(budget_bytes=2 << 30, max_limit=10**7, max_active=4, chunks=1, tune=tune)
    tickets = [srv.submit(j) for j in jobs]
    for t in tickets:
        assert srv.wait(t, 120.0).state == 2
    for job, t in zip(jobs, tickets):
        b, c = srv.fetch(t)
        torch.cuda.synchronize()
        a_b, a_c = _alone(job, tune)
        assert np.array_equal(_np(b), a_b) and np.array_equal(_np(c), a_c), job
        srv.release(t)
    w_b, w_c = coracle.sieve_job(odd)
    a_b, a_c = _alone(odd, tune)
    assert np.array_equal(a_b, w_b) and np.array_equal(a_c, w_c)
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["bytes_iterations"] < st["iterations"]
    srv.close()


def test_budget_forces_queueing_and_results_hold():
    """A budget that fits about one job at a time: jobs wait for memory, results are unchanged."""
    jobs = [W.Job(307, 2, 12345 + 1000 * i, 4000, 2500, 10**7) for i in range(4)]
    tune = cs.Tune(large_mode=cs.LARGE_THREE_GAP)
    srv = cs.Server(budget_bytes=400 << 20, max_limit=10**7, max_active=8, chunks=2, tune=tune)
    tickets = [srv.submit(j) for j in jobs]
    peak = 0
    while True:
        st = srv.stats()
        peak = max(peak, st["bytes_in_use"])
        if st["completed"] == len(jobs):
            break
        time.sleep(0.002)
    assert peak <= 400 << 20
    for job, t in zip(jobs, tickets):
        info = srv.poll(t)
        assert info.state == 2
        b, c = srv.fetch(t)
        torch.cuda.synchronize()
        a_b, a_c = _alone(job, tune)
        assert np.array_equal(_np(b), a_b) and np.array_equal(_np(c), a_c)
        srv.release(t)
    srv.close()


def test_oversized_job_is_rejected():
    srv = cs.Server(budget_bytes=64 << 20, max_limit=10**7, max_active=2)
    with pytest.raises(cs.CsError) as e:
        srv.submit(W.Job(307, 2, 1, 4000, 2500, 2 * 10**7))       # limit above max_limit
    assert e.value.status == -2
    with pytest.raises(cs.CsError) as e:
        srv.submit(W.Job(307, 1, 1, 900000, 60000, 10**7))        # outputs beyond the budget
    assert e.value.status == -2
    srv.close()

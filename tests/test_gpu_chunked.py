"""The chunked sieve (cs_sieve_chunked): the prime range taken in chunks of a fixed number of
integers, each with its own prime table and K mod p, gives exactly cs_sieve's bitmap and
counts, on jobs whose limits span several chunks, in both enumerations of the large primes.
Windows of the prime range near 2^41 and 2^42 (cs_sieve_chunked_range) against the oracle."""
import functools

import numpy as np
import pytest

import workloads as W
from oracle import coracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2012_03771_amd as cs  # noqa: E402


def _say(*a):
    print(*a, flush=True)


JOBS = [W.Job(61, 6, 1000, 3000, 500, 10**8), W.Job(211, 2 * 3 * 5 * 7 * 101, 1, 6000, 2000, 2 * 10**8),
        W.Job(503, 210, 10**6, 10**4, 7000, 10**8)]


@pytest.mark.parametrize("job", JOBS, ids=lambda j: "P%d_d%d_m%d+%d_sl%d_L%d" % j.as_tuple())
@pytest.mark.parametrize("mode", [cs.LARGE_G, cs.LARGE_THREE_GAP], ids=["g", "three_gap"])
def test_chunked_equals_whole(job, mode):
    tune = cs.Tune(large_mode=mode)
    _say("chunked", job, mode)
    b0, c0, ws0 = cs.sieve(job, tune)
    d0 = cs.diag_read(ws0)
    for span in (1 << 25, 3 << 25):
        b1, c1, ws1 = cs.sieve_chunked(job, span, tune)
        d1 = cs.diag_read(ws1)
        assert torch.equal(b0, b1) and torch.equal(c0, c1), span
        assert d1.n_primes == d0.n_primes and d1.large_hits == d0.large_hits
        assert d1.small_marks == d0.small_marks
        del b1, c1, ws1


def test_chunked_paper_scale():
    """953#/210, primes to 1e10, in five chunks of 2^31 integers (a workspace of 5.3 GiB instead
    of the 13.6 GiB of the whole sieve with K mod p tables for every prime): the same bitmap and
    counts as the whole sieve."""
    job = W.PAPER_SCALE
    tune = cs.Tune(large_mode=cs.LARGE_THREE_GAP)
    _say("chunked paper scale")
    lay = cs.plan_chunked(job, 1 << 31, tune)
    assert lay.ws_bytes < cs.plan(job, cs.Tune(large_mode=cs.LARGE_THREE_GAP, kmod=cs.KMOD_TABLE)).ws_bytes / 2
    b0, c0, ws0 = cs.sieve(job, tune)
    h0, k0 = b0.cpu(), c0.cpu()
    n0 = cs.diag_read(ws0).n_primes
    del b0, c0, ws0
    torch.cuda.empty_cache()
    b1, c1, ws1 = cs.sieve_chunked(job, 1 << 31, tune)
    assert cs.diag_read(ws1).n_primes == n0 == 455052511
    assert torch.equal(b1.cpu(), h0) and torch.equal(c1.cpu(), k0)


def test_chunked_ranges_compose():
    """[2, limit] split into three ranges (ORed bitmaps, summed counts) equals the whole chunked
    sieve; an empty range (p_hi < p_lo) changes nothing."""
    job = W.Job(211, 2 * 3 * 5 * 7 * 101, 1, 6000, 2000, 2 * 10**8)
    tune = cs.Tune(large_mode=cs.LARGE_THREE_GAP)
    span = 1 << 25
    _say("chunked ranges", job)
    b0, c0, _ = cs.sieve_chunked(job, span, tune)
    lay = cs.plan_chunked(job, span, tune)
    b1 = torch.zeros((lay.n_m, lay.row_words), dtype=torch.int32, device="cuda")
    c1 = torch.zeros((lay.n_m,), dtype=torch.int32, device="cuda")
    ws = torch.empty((lay.ws_bytes,), dtype=torch.uint8, device="cuda")
    for lo, hi in ((0, 10**5), (10**5 + 1, 3 * span + 17), (3 * span + 18, job.limit), (50, 49)):
        cs.sieve_chunked_range(job, span, lo, hi, b1, c1, ws, tune)
    assert torch.equal(b0, b1) and torch.equal(c0, c1)


# windows of 2^24 integers of the prime range, up to the largest limit (2^42 - 1); the second
# one straddles the chunk boundary at 2^41.  A prime near 2^42 divides some m K + X of a row
# with probability (number of columns) / p, so the job is wide (102,988 columns, 16,000 rows)
# to give a few hundred hits per window.
WINDOW_JOB = W.Job(61, 6, 10**6, 48000, 131000, 2**42 - 1)
WINDOWS = [(2**42 - 2**24, 2**42 - 1), (2**41 - 2**23, 2**41 + 2**23)]


@functools.lru_cache(maxsize=None)
def _window_oracle(lo, hi):
    job = WINDOW_JOB
    m_all = coracle.rows(job.d, job.m_start, job.m_inc)
    return coracle.sieve_rows(job.P, job.d, job.sl, m_all, lo, hi, mode=coracle.CACHED)


@pytest.mark.parametrize("lo,hi", WINDOWS, ids=["below_2^42", "across_2^41"])
@pytest.mark.parametrize("mode", [cs.LARGE_G, cs.LARGE_THREE_GAP], ids=["g", "three_gap"])
def test_window_near_2_42(lo, hi, mode):
    """Every prime of the window, with its prime table sieved from base primes beyond 2^20 and
    K mod p and m K mod p near 2^42: bitmap and counts of every row equal the oracle's."""
    job = WINDOW_JOB
    tune = cs.Tune(large_mode=mode)
    span = 1 << 25
    _say("window", lo, hi, mode)
    lay = cs.plan_chunked(job, span, tune)
    b = torch.zeros((lay.n_m, lay.row_words), dtype=torch.int32, device="cuda")
    c = torch.zeros((lay.n_m,), dtype=torch.int32, device="cuda")
    ws = torch.empty((lay.ws_bytes,), dtype=torch.uint8, device="cuda")
    cs.sieve_chunked_range(job, span, lo, hi, b, c, ws, tune)
    torch.cuda.synchronize()
    want_b, want_c = _window_oracle(lo, hi)
    _say("oracle hits", int(want_c.sum()))
    got_b = b.cpu().numpy().view(np.uint32)
    got_c = c.cpu().numpy().view(np.uint32)
    assert want_c.sum() > 100
    assert np.array_equal(got_c, want_c), (int(got_c.sum()), int(want_c.sum()))
    assert np.array_equal(got_b, want_b)

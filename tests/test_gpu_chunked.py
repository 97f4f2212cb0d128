"""The chunked sieve (cs_sieve_chunked): the prime range taken in chunks of a fixed number of
integers, each with its own prime table and K mod p, gives exactly cs_sieve's bitmap and
counts, on jobs whose limits span several chunks, in both enumerations of the large primes."""
import numpy as np
import pytest

import workloads as W

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
    of 13.6 GiB): the same bitmap and counts as the whole sieve."""
    job = W.PAPER_SCALE
    tune = cs.Tune(large_mode=cs.LARGE_THREE_GAP)
    _say("chunked paper scale")
    lay = cs.plan_chunked(job, 1 << 31, tune)
    assert lay.ws_bytes < cs.plan(job, tune).ws_bytes / 2
    b0, c0, ws0 = cs.sieve(job, tune)
    h0, k0 = b0.cpu(), c0.cpu()
    n0 = cs.diag_read(ws0).n_primes
    del b0, c0, ws0
    torch.cuda.empty_cache()
    b1, c1, ws1 = cs.sieve_chunked(job, 1 << 31, tune)
    assert cs.diag_read(ws1).n_primes == n0 == 455052511
    assert torch.equal(b1.cpu(), h0) and torch.equal(c1.cpu(), k0)

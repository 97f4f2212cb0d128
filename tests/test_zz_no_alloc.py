"""cs_sieve_noalloc (the whole sieve with the library's own static device workspace) against
cs_sieve, through the C ABI: two calls in a row on one stream, the second with a smaller job, each
bit-identical to cs_sieve on the same job; and a job whose workspace exceeds the array is refused
before anything is enqueued."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2012_03771_amd as cs  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _reference(job, tune):
    bitmap, counts, ws = cs.sieve(job, tune)
    torch.cuda.synchronize()
    out = bitmap.cpu().numpy().view(np.uint32).copy(), counts.cpu().numpy().view(np.uint32).copy()
    del bitmap, counts, ws
    return out


@pytest.mark.parametrize("tune", [None, cs.Tune(large_mode=cs.LARGE_THREE_GAP),
                                  cs.Tune(large_mode=cs.LARGE_THREE_GAP, scatter=cs.SCATTER_ATOMIC)],
                         ids=["g_bytes", "three_gap_bytes", "three_gap_atomic"])
def test_noalloc_equals_sieve_on_two_calls(tune):
    s = torch.cuda.current_stream()
    cap = cs.scratch_bytes()
    assert cap == 256 << 20
    jobs = [W.MEDIUM, W.SMALL]                       # the second call is the smaller job
    assert cs.plan(jobs[0], tune).ws_bytes > cs.plan(jobs[1], tune).ws_bytes
    outs = []
    for job in jobs:
        lay = cs.plan(job, tune)
        assert lay.ws_bytes <= cap
        _say("noalloc", job, tune)
        bitmap = torch.full((lay.n_m, lay.row_words), -1, dtype=torch.int32, device="cuda")
        counts = torch.full((lay.n_m,), -1, dtype=torch.int32, device="cuda")
        cs.sieve_noalloc_into(job, bitmap, counts, tune, s)
        outs.append((job, bitmap, counts))
    torch.cuda.synchronize()
    for job, bitmap, counts in outs:
        want_b, want_c = _reference(job, tune)
        assert np.array_equal(bitmap.cpu().numpy().view(np.uint32), want_b), f"{job}: bitmap differs"
        assert np.array_equal(counts.cpu().numpy().view(np.uint32), want_c), f"{job}: counts differ"


def test_noalloc_refuses_a_workspace_beyond_the_array():
    lay = cs.plan(W.PAPER_SCALE)
    assert lay.ws_bytes > cs.scratch_bytes()
    bitmap = torch.zeros((1, 1), dtype=torch.int32, device="cuda")
    with pytest.raises(cs.CsError) as e:
        cs.sieve_noalloc_into(W.PAPER_SCALE, bitmap, bitmap[0], None)
    assert e.value.status == -2

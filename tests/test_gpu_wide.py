"""The exact 64-bit residue path (primes from 2^42, Section 3.3's p < 2^64) on the GPU.

* Forced onto it from 2^20 (cs_tune.wide_log2), every large prime of real jobs takes the
  64-bit K mod p, Euclidean pass, Eq. 5 descent and walk: outputs must equal the fp64 path's.
* K mod p for primes near 2^42, 2^50 and 2^62 against Python's bignum K % p.
* Windows of the prime range near 2^50 and just below 2^63, with jobs placed where primes of the
  window divide their intervals (tests/golden/make_golden.py, wide()): every row against the
  oracle's direct sieve, through the chunked sieve whose chunk there needs the level-2 base
  primes up to 3.04e9."""
import math
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


def _say(*a):
    print(*a, flush=True)


def _run(job, tune):
    b, c, ws = cs.sieve(job, tune)
    torch.cuda.synchronize()
    d = cs.diag_read(ws)
    out = b.cpu().numpy().view(np.uint32).copy(), c.cpu().numpy().view(np.uint32).copy(), d
    del b, c, ws
    torch.cuda.empty_cache()
    return out


JOBS = [W.MEDIUM, W.Job(61, 6, 1000, 3000, 500, 10**7), W.Job(211, 210, 10**12, 20000, 4000, 5 * 10**8),
        W.Job(401, 1, 7, 5000, 3000, 2 * 10**8)]


@pytest.mark.parametrize("job", JOBS, ids=lambda j: "P%d_d%d" % (j.P, j.d))
@pytest.mark.parametrize("mode,scatter", [(cs.LARGE_G, cs.SCATTER_AUTO), (cs.LARGE_THREE_GAP, cs.SCATTER_AUTO),
                                          (cs.LARGE_THREE_GAP, cs.SCATTER_LIST),
                                          (cs.LARGE_THREE_GAP, cs.SCATTER_ATOMIC)],
                         ids=["g", "three_gap", "three_gap_list", "three_gap_atomic"])
def test_forced_64_bit_path_equals_fp64_path(job, mode, scatter):
    _say("forced wide", job, mode, scatter)
    b0, c0, d0 = _run(job, cs.Tune(large_mode=mode, scatter=scatter))
    b1, c1, d1 = _run(job, cs.Tune(large_mode=mode, scatter=scatter, wide_log2=20))
    assert d1.error_flags == 0
    assert np.array_equal(b0, b1) and np.array_equal(c0, c1)
    assert d1.large_hits + d1.small_marks == d0.large_hits + d0.small_marks
    assert d1.large_raw_hits == d0.large_raw_hits or d1.large_primes != d0.large_primes


def test_forced_64_bit_path_paper_scale():
    job = W.PAPER_SCALE
    tune = cs.Tune(large_mode=cs.LARGE_THREE_GAP)
    _say("forced wide paper")
    b0, c0, d0 = _run(job, tune)
    b1, c1, d1 = _run(job, cs.Tune(large_mode=cs.LARGE_THREE_GAP, wide_log2=20))
    assert d1.error_flags == 0
    assert np.array_equal(c0, c1) and np.array_equal(b0, b1)


def _is_prime64(n: int) -> bool:
    """Miller-Rabin with the first twelve prime bases: exact for every n < 3.3e24."""
    if n < 2:
        return False
    bases = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for q in bases:
        if n % q == 0:
            return n == q
    dd, s = n - 1, 0
    while dd % 2 == 0:
        dd //= 2
        s += 1
    for a in bases:
        x = pow(a, dd, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


@pytest.mark.parametrize("centre", [(1 << 42) - 10**6, 1 << 42, 1 << 50, (1 << 62) + (1 << 40), (1 << 63) - (1 << 22)])
def test_kmod_of_64_bit_primes_against_bignum(centre):
    P, d = 953, 210
    K = math.prod(q for q in range(2, P + 1) if all(q % r for r in range(2, int(q ** 0.5) + 1))) // d
    ps = np.array([n for n in range(centre | 1, centre + 40000, 2) if _is_prime64(n)][:600], dtype=np.uint64)
    assert len(ps) > 100
    got = cs.kmod(P, d, torch.from_numpy(ps.astype(np.int64)).cuda()).cpu().numpy().astype(np.uint64)
    want = np.array([K % int(p) for p in ps], dtype=np.uint64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("mode", [cs.LARGE_G, cs.LARGE_THREE_GAP], ids=["g", "three_gap"])
@pytest.mark.parametrize("name", ["w50", "w63"])
def test_window_of_64_bit_primes_against_oracle(name, mode):
    g = load("wide_windows.npz")
    job = W.Job(*[int(x) for x in g[f"{name}_job"]])
    p_lo, p_hi, q, n_pr = [int(x) for x in g[f"{name}_window"]]
    span = 1 << 25
    tune = cs.Tune(large_mode=mode)
    lay = cs.plan_chunked(job, span, tune)
    _say(name, job, p_lo, p_hi, lay.ws_bytes / 2**30)
    bitmap = torch.zeros((lay.n_m, lay.row_words), dtype=torch.int32, device="cuda")
    counts = torch.zeros((lay.n_m,), dtype=torch.int32, device="cuda")
    ws = torch.empty((lay.ws_bytes,), dtype=torch.uint8, device="cuda")
    cs.sieve_chunked_range(job, span, p_lo, p_hi, bitmap, counts, ws, tune)
    torch.cuda.synchronize()
    d = cs.diag_read(ws)
    b = bitmap.cpu().numpy().view(np.uint32)
    c = counts.cpu().numpy().view(np.uint32)
    assert d.error_flags == 0
    assert d.large_primes == n_pr                   # the window's primes, from the oracle's sieve
    assert int(c.sum()) == int(g[f"{name}_counts"].sum()) >= 39
    assert np.array_equal(c, g[f"{name}_counts"]) and np.array_equal(b, g[f"{name}_bits"])
    del bitmap, counts, ws
    torch.cuda.empty_cache()

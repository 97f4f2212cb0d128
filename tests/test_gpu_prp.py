"""GPU parity of the probable-prime stage: cs_prp_numbers against the oracle's strong test on
numbers of every limb count, and cs_surround on sieved rows against the oracle's sequential
search (same candidates, same order), including the paper's two record gaps."""
import math
import os
import random
import sys

import numpy as np
import pytest

import workloads as W
from oracle import coracle, plain, prp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2012_03771_amd as cs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _say(*a):
    print(*a, flush=True)


def _limbs(ns, n_limbs):
    arr = np.stack([prp.limbs(n, n_limbs) for n in ns]).view(np.int32)
    return torch.from_numpy(arr).cuda()


def _gpu_prp(ns, n_limbs):
    out = cs.prp_numbers(_limbs(ns, n_limbs))
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(bool)


_SMALL_PRODUCT = plain.primorial(3000)


def _next_prp(n):
    """Smallest probable prime >= n (numbers with a factor below 3000 skipped by one gcd)."""
    import math
    n |= 1
    while math.gcd(n, _SMALL_PRODUCT) > 1 or not prp.sprp2(n):
        n += 2
    return n


SPECIAL = [0, 1, 2, 3, 4, 5, 9, 15, 2047, 3277, 4033, 4681, 8321, 561, 1105, 1729, 65537, 2**31 - 1,
           2**32 + 15, 2**61 - 1, 2**67 - 1, 2**64 - 59, 2**89 - 1, (2**61 - 1) * (2**89 - 1),
           2**127 - 1, 3 * 2**100 + 1, 2**128 + 1, 2**521 - 1, 2**607 - 1, 2**1279 - 1]
# the ends of the paper's two record gaps (Section 1), and their neighbours
_R1 = 100054841 * plain.K_of(953, 210)
_R2 = 164065661 * plain.K_of(1019, 210)
SPECIAL += [_R1 - 9670, _R1 + 25638, _R2 - 18566, _R2 + 18136, _R1 - 9672, _R1 + 25640, _R2 - 18564,
            (2**89 - 1) * (_R1 - 9670)]


@pytest.mark.parametrize("n_limbs", [1, 2, 3, 4, 7, 8, 12, 16, 20, 24, 28, 32, 36, 40, 42, 44, 48, 52, 56, 60, 64])
def test_prp_numbers_against_oracle(n_limbs):
    _say("prp_numbers n_limbs", n_limbs)
    rng = random.Random(n_limbs)
    bits = 32 * n_limbs
    ns = [x for x in SPECIAL if x.bit_length() <= bits]
    for _ in range(300 if n_limbs <= 16 else 120):
        b = rng.randint(max(2, bits - 40), bits)
        ns.append(rng.getrandbits(b) | 1)
    for _ in range(40 if n_limbs <= 8 else 12 if n_limbs <= 24 else 2):   # probable primes near random points
        b = rng.randint(max(3, bits - 8), bits - 1)
        p = _next_prp(rng.getrandbits(b) | (1 << (b - 1)))
        if p.bit_length() <= bits:
            ns.append(p)
            q = _next_prp(p + 2)
            if p * q < 2**bits:
                ns.append(p * q)
    got = _gpu_prp(ns, n_limbs)
    want = np.array([prp.sprp2(n) for n in ns])
    bad = [ns[i] for i in np.nonzero(got != want)[0]]
    assert not bad, bad[:4]
    assert want.sum() >= 2


def test_prp_numbers_even_and_edge_counts():
    ns = list(range(0, 200))
    got = _gpu_prp(ns, 1)
    assert np.array_equal(got, np.array([prp.sprp2(n) for n in ns]))
    empty = cs.prp_numbers(torch.zeros((0, 3), dtype=torch.int32, device="cuda"))
    assert empty.numel() == 0
    with pytest.raises(cs.CsError):
        cs.prp_numbers(torch.zeros((4, 65), dtype=torch.int32, device="cuda"))


def _sieve_and_surround(job, rows_idx=None):
    b, c, ws = cs.sieve(job)
    ms = cs.rows(job)
    if rows_idx is not None:
        b = b[torch.as_tensor(rows_idx, device="cuda")].contiguous()
        ms = ms[rows_idx]
    m_dev = torch.from_numpy(ms.astype(np.int64)).cuda()
    out, stats = cs.surround(job, b, m_dev)
    return b.cpu().numpy().view(np.uint32), ms, out.cpu().numpy(), stats


def _oracle_rows(job, ms):
    bits, _ = coracle.sieve_rows(job.P, job.d, job.sl, ms, 2, job.limit)
    nx = len(plain.columns(job.P, job.d, job.sl))
    ub = plain.unpack(bits, nx)
    return bits, prp.surround_rows(job.P, job.d, ms, job.sl, ub)


@pytest.mark.parametrize("job", [W.SMALL, W.Job(61, 6, 1000, 400, 300, 10**5), W.Job(131, 30, 7, 300, 900, 2 * 10**5),
                                 W.Job(13, 2, 1, 200, 30, 1000), W.Job(307, 2, 12345, 200, 2500, 10**6)],
                         ids=["small_211", "p61", "p131", "p13_tiny", "p307"])
def test_surround_every_row_against_oracle(job):
    _say("surround", job)
    gb, ms, out, stats = _sieve_and_surround(job)
    ob, want = _oracle_rows(job, ms)
    assert np.array_equal(gb, ob)                          # same sieve input on both sides
    want = np.array(want, dtype=np.int64).reshape(-1, 4)
    assert np.array_equal(out.astype(np.int64), want), np.nonzero((out != want).any(1))[0][:5]
    assert stats.tests >= want[:, 2:].sum() and stats.rounds >= 1 and stats.test_ms > 0


def test_surround_paper_scale_sampled_rows():
    """953#/210, m in [1e8, 1e8 + 1e6), sl = 20000, sieved to 1e10 on the GPU: for 24 sampled rows
    the nearest probable primes equal the oracle's sequential search over all columns (the sieve
    only removes composites, so the answer does not depend on it)."""
    job = W.PAPER_SCALE
    idx = np.array(W.sample_rows(cs.plan(job).n_m, 24, seed=7))
    _say("paper-scale rows", idx[:4], "...")
    _, ms, out, stats = _sieve_and_surround(job, idx)
    want = prp.surround_rows(job.P, job.d, ms, job.sl, None, trial=2000)
    for i, (p, n, tp, tn) in enumerate(want):
        assert out[i, 0] == p and out[i, 1] == n, (i, int(ms[i]), out[i], (p, n))
        assert out[i, 2] >= 1 and out[i, 3] >= 1
    assert stats.limbs == 44


@pytest.mark.parametrize("which", [0, 1], ids=["gap_35308", "gap_36702"])
def test_record_gaps_found_on_the_gpu(paper_values, which):
    """The two record gaps of Section 1: sieve the row of m on the GPU to 1e9, search outward."""
    g = paper_values["record_gaps"]["gaps"][which]
    prev, nxt = g["x_prev"], g["x_prev"] + g["gap"]
    sl = max(-prev, nxt) + 100
    job = W.Job(g["P"], g["d"], g["m"], 1, sl, 10**9)
    _say("record", job)
    _, ms, out, stats = _sieve_and_surround(job)
    assert out[0, 0] == prev and out[0, 1] == nxt
    N = g["m"] * plain.K_of(g["P"], g["d"])
    merit = (nxt - prev) / math.log(N + prev)
    assert round(merit, 3) == g["merit"]


def test_surround_empty_sides_and_validation():
    # sl too small for any probable prime near a primorial multiple: both sides report 0
    job = W.Job(211, 210, 1, 50, 30, 10**5)
    gb, ms, out, stats = _sieve_and_surround(job)
    _, want = _oracle_rows(job, ms)
    assert np.array_equal(out.astype(np.int64), np.array(want, dtype=np.int64).reshape(-1, 4))
    # m outside the job's range is reported by the device check
    b, c, ws = cs.sieve(job)
    bad_m = torch.full((b.shape[0],), 10**6, dtype=torch.int64, device="cuda")
    with pytest.raises(cs.CsError):
        cs.surround(job, b, bad_m)


def test_advisor_sieve_limit_and_interval():
    """Section 4: the sieve-limit advice stops where the tests saved per second of sieving fall
    below the probable-prime rate; the interval check counts rows whose surrounding primes lie
    beyond sl."""
    from paper_2012_03771_amd import advisor as A
    job = W.Job(503, 210, 10**6, 2000, 7000, 10**8)
    rate = A.prp_rate(job, n_tests=4096)
    assert rate > 1e4
    adv = A.advise_sieve_limit(job, prp_tests_per_s=rate)
    assert adv.steps[0].p_lo == 1 and adv.steps[-1].p_hi == job.limit
    assert all(s.ms > 0 for s in adv.steps)
    assert all(a.p_hi == b.p_lo for a, b in zip(adv.steps, adv.steps[1:]))
    saved = [s.tests_saved for s in adv.steps[1:]]
    assert all(x > 0 for x in saved)
    # the advice is the end of the last range that beat the rate
    keep = [s.p_hi for s in adv.steps if s.p_lo == 1 or s.saved_per_s >= rate]
    assert adv.limit == keep[-1]
    assert A.advise_sieve_limit(job, prp_tests_per_s=0.0).limit == job.limit
    assert A.advise_sieve_limit(job, prp_tests_per_s=float("inf")).limit == adv.steps[0].p_hi
    # interval: sl = 7000 > 10 log N for 503#/210: almost every row finds both primes
    ok = A.check_interval(job, rows=128)
    assert ok.rows == 128 and not ok.warn
    # sl below 6 log N: many rows reach beyond it
    narrow = A.check_interval(W.Job(503, 210, 10**6, 2000, 300, 10**8), rows=128)
    assert narrow.warn and narrow.beyond > 10
    _, want = _oracle_rows(W.Job(503, 210, 10**6, 300, 300, 10**8), cs.rows(W.Job(503, 210, 10**6, 300, 300, 10**8))[:32])
    assert sum(1 for p, n, _, _ in want if p == 0 or n == 0) > 0


# ------------------------------------------------------------------------------------------
# The strong Lucas test and BPSW (cs_prp_test)
# ------------------------------------------------------------------------------------------
LUCAS_SPECIAL = [5459, 5777, 10877, 16109, 18971, 22499, 24569, 25199, 40309, 58519, 75077, 97439,
                 25, 49, 121, 169, 3**20, 65521**2, 7, 11, 13, 97, 5 * 7 * 11]


def _gpu_test(ns, n_limbs, test):
    out = cs.prp_test(_limbs(ns, n_limbs), test)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(bool)


def test_lucas_and_bpsw_small_numbers():
    """Every n below 20,000 and the strong Lucas pseudoprimes below 10^5, as one-limb numbers."""
    ns = list(range(0, 20000)) + LUCAS_SPECIAL
    _say("lucas small", len(ns))
    for test, ref in ((cs.PRP_LUCAS, prp.strong_lucas), (cs.PRP_BPSW, prp.bpsw), (cs.PRP_SPRP2, prp.sprp2)):
        got = _gpu_test(ns, 1, test)
        want = np.array([ref(n) for n in ns])
        bad = [ns[i] for i in np.nonzero(got != want)[0]]
        assert not bad, (test, bad[:6])


@pytest.mark.parametrize("n_limbs", [2, 3, 8, 12, 16, 20, 44, 64])
def test_lucas_and_bpsw_against_oracle(n_limbs):
    _say("lucas n_limbs", n_limbs)
    rng = random.Random(1000 + n_limbs)
    bits = 32 * n_limbs
    ns = [x for x in SPECIAL + LUCAS_SPECIAL if x.bit_length() <= bits and (x < 2**32 or math.isqrt(x)**2 != x)]
    for _ in range(60 if n_limbs <= 16 else 16):
        b = rng.randint(max(2, bits - 40), bits)
        ns.append(rng.getrandbits(b) | 1)
    for _ in range(12 if n_limbs <= 16 else 3):            # probable primes and products of two
        b = rng.randint(max(3, bits // 2 - 8), bits // 2 - 1)
        p = _next_prp(rng.getrandbits(b) | (1 << (b - 1)))
        q = _next_prp(p + 2)
        ns += [p, p * q]
    ns = [n for n in ns if n.bit_length() <= bits]
    for test, ref in ((cs.PRP_LUCAS, prp.strong_lucas), (cs.PRP_BPSW, prp.bpsw)):
        got = _gpu_test(ns, n_limbs, test)
        want = np.array([ref(n) for n in ns])
        bad = [ns[i] for i in np.nonzero(got != want)[0]]
        assert not bad, (test, bad[:4])
        assert want.sum() >= 2
    with pytest.raises(cs.CsError):
        cs.prp_test(_limbs(ns[:2], n_limbs), 3)


def test_surround_searches_past_a_base2_pseudoprime():
    """N = 68 * 5# = 2040 sieved to 20: above N the unmarked numbers are 2047 = 23 * 89, a strong
    pseudoprime to base 2, then the prime 2053.  BPSW rejects 2047, so the side searches on (a
    second Lucas pass) and stops at X = 13; below N, 2039 (X = -1) is prime."""
    job = W.Job(5, 1, 68, 1, 20, 20)
    gb, ms, out, stats = _sieve_and_surround(job)
    ob, want = _oracle_rows(job, ms)
    assert np.array_equal(gb, ob)
    assert [tuple(int(v) for v in r) for r in out] == [tuple(w) for w in want] == [(-1, 13, 1, 2)]
    # each pass tests every side that holds a probable prime: 2 in the first, 2 again in the second
    assert stats.lucas_passes == 2 and stats.lucas_tests == 4 and stats.lucas_ms > 0

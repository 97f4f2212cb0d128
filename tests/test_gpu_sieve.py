"""GPU parity of the HIP path against the CPU oracle, element by element, through the C ABI.

Every expected value comes from oracle/ (run here on the same seeded jobs) or from the paper."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import coracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2012_03771_amd as cs  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(job, tune=None):
    bitmap, counts, ws = cs.sieve(job, tune)
    torch.cuda.synchronize()
    diag = cs.diag_read(ws)
    return bitmap.cpu().numpy().view(np.uint32), counts.cpu().numpy().view(np.uint32), diag, ws


def _oracle(job, mode=coracle.CACHED, m_rows=None):
    if m_rows is None:
        return coracle.sieve_job(job, mode=mode)
    return coracle.sieve_rows(job.P, job.d, job.sl, m_rows, 2, job.limit, mode=mode)


def _assert_same(job, got_b, got_c, want_b, want_c, rows=None):
    if rows is not None:
        got_b, got_c = got_b[rows], got_c[rows]
    if not np.array_equal(got_b, want_b) or not np.array_equal(got_c, want_c):
        bad = np.nonzero((got_b != want_b).any(axis=1) | (got_c != want_c))[0]
        r = bad[0]
        raise AssertionError(f"{job}: {len(bad)} rows differ, first row {r}: counts gpu={got_c[r]} "
                             f"oracle={want_c[r]}, words differing={int((got_b[r] != want_b[r]).sum())}")


# ------------------------------------------------------------------------------------------
# prime table and K mod p
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("limit", [2, 3, 10, 100, 1000, 2**19 - 1, 2**19, 2**19 + 1, 3 * 2**19 + 7, 10**6,
                                   10**7, 2 * 10**8 + 7])
def test_prime_table_matches_oracle(limit):
    _say("primes", limit)
    got, n = cs.primes(limit)
    want = coracle.primes_range(2, limit)
    assert n == len(want)
    assert np.array_equal(got.cpu().numpy().astype(np.uint64), want)


@pytest.mark.parametrize("x", [10**8, 4 * 10**9, 10**10])
def test_prime_counts_printed_in_paper(paper_values, x):
    _say("pi", x)
    _, n = cs.primes(x)
    assert n == paper_values["prime_counts"][str(x)]


@pytest.mark.parametrize("P,d", [(211, 210), (503, 210), (953, 210), (1019, 1), (11, 2), (5, 30)])
def test_kmod_matches_bignum(P, d):
    _say("kmod", P, d)
    ps = np.concatenate([coracle.primes_range(2, 2 * 10**5),
                         coracle.primes_range(10**10 - 10**5, 10**10),
                         coracle.primes_range(2**39 - 2**14, 2**39),
                         coracle.primes_range(2**42 - 2**13, 2**42 - 1)])
    dev = torch.from_numpy(ps.astype(np.int64)).cuda()
    got = cs.kmod(P, d, dev).cpu().numpy().astype(np.uint64)
    K = 1
    for q in coracle.primes_range(2, P):
        K *= int(q)
    K //= d
    want = np.array([K % int(p) for p in ps], dtype=np.uint64)
    assert np.array_equal(got, want)


# ------------------------------------------------------------------------------------------
# whole jobs
# ------------------------------------------------------------------------------------------
TINY = W.tiny_jobs(seed=5, n=40, max_P=31) + [W.Job(11, d, 7, 40, 60, 3000) for d in (1, 2, 6, 30, 210)]


@pytest.mark.parametrize("job", TINY, ids=lambda j: "P%d_d%d_m%d+%d_sl%d_L%d" % j.as_tuple())
def test_tiny_jobs(job):
    want_b, want_c = _oracle(job, mode=coracle.DIRECT)
    for tune in (None, cs.Tune(thr=1), cs.Tune(thr=1, large_mode=cs.LARGE_THREE_GAP),
                 cs.Tune(thr=10**9), cs.Tune(thr=1, scatter=cs.SCATTER_ATOMIC),
                 cs.Tune(thr=1, scatter=cs.SCATTER_BYTES), cs.Tune(thr=1, scatter=cs.SCATTER_LIST, list_chunks=1),
                 cs.Tune(thr=1, large_mode=cs.LARGE_THREE_GAP, scatter=cs.SCATTER_LIST, list_chunks=2),
                 cs.Tune(thr=1, large_mode=cs.LARGE_THREE_GAP, scatter=cs.SCATTER_LIST)):
        b, c, _, _ = _run(job, tune)
        _assert_same(job, b, c, want_b, want_c)


MIXED = [W.Job(61, 6, 1000, 3000, 500, 10**6), W.Job(97, 30, 10**6, 20000, 1200, 5 * 10**6),
         W.Job(131, 1, 7, 5000, 900, 2 * 10**6), W.Job(307, 2, 12345, 4000, 2500, 10**7),
         W.Job(401, 210, 99, 30000, 3000, 10**7),
         # d with a large prime factor (the form of the paper's amortized-runtime table, d = 7#*q):
         # rows come from the dense m -> row table rather than the d-residue table
         W.Job(211, 2 * 3 * 5 * 7 * 101, 1, 6000, 2000, 10**6), W.Job(409, 2 * 3 * 5 * 7 * 401, 777, 20000, 1500, 3 * 10**6)]


@pytest.mark.parametrize("job", MIXED, ids=lambda j: "P%d_d%d_m%d+%d_sl%d_L%d" % j.as_tuple())
def test_mixed_jobs_both_modes(job):
    _say("mixed", job)
    want_b, want_c = _oracle(job)
    for tune in (None, cs.Tune(large_mode=cs.LARGE_THREE_GAP), cs.Tune(thr=1, hits_per_item=8),
                 cs.Tune(tile_rows=3, small_slices=5), cs.Tune(scatter=cs.SCATTER_ATOMIC),
                 cs.Tune(large_mode=cs.LARGE_THREE_GAP, scatter=cs.SCATTER_ATOMIC, thr=1),
                 cs.Tune(scatter=cs.SCATTER_BYTES), cs.Tune(thr=1, hits_per_item=8, scatter=cs.SCATTER_LIST, list_chunks=3),
                 cs.Tune(large_mode=cs.LARGE_THREE_GAP, thr=1, hits_per_item=8)):
        b, c, diag, _ = _run(job, tune)
        _assert_same(job, b, c, want_b, want_c)
        assert diag.small_marks + diag.large_hits == int(want_c.sum())


def test_small_211_job():
    job = W.SMALL
    want_b, want_c = _oracle(job)
    for tune in (None, cs.Tune(thr=1), cs.Tune(large_mode=cs.LARGE_THREE_GAP), cs.Tune(thr=2 * 10**6)):
        b, c, diag, _ = _run(job, tune)
        _assert_same(job, b, c, want_b, want_c)
        assert diag.n_primes == 78498


def test_medium_503_sampled_rows():
    job = W.MEDIUM
    lay = cs.plan(job)
    rows = W.sample_rows(lay.n_m, 24, seed=2)
    ms = cs.rows(job)[rows]
    want_b, want_c = _oracle(job, m_rows=ms)
    for tune in (None, cs.Tune(large_mode=cs.LARGE_THREE_GAP)):
        b, c, diag, _ = _run(job, tune)
        _assert_same(job, b, c, want_b, want_c, rows=rows)
        u = cs.unpack_bits(b, lay.n_x)
        assert np.all(c >= u.sum(axis=1))


def test_range_calls_compose():
    """cs_prepare + cs_sieve_range over a split of [2, limit] equals cs_sieve."""
    job = W.Job(211, 210, 5000, 3000, 4000, 3 * 10**6)
    ref_b, ref_c, _, _ = _run(job)
    lay, bitmap, counts, ws = cs.binding.alloc_outputs(job)
    bitmap.zero_()
    counts.zero_()
    cs.prepare(job, ws)
    edges = [2, 97, 8000, 10**5, 400000, 1234567, job.limit]
    for a, b in zip(edges[:-1], edges[1:]):
        cs.sieve_range(job, a, b - 1 if b != job.limit else b, bitmap, counts, ws)
    torch.cuda.synchronize()
    assert np.array_equal(bitmap.cpu().numpy().view(np.uint32), ref_b)
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), ref_c)


@pytest.mark.parametrize("job,mult", [
    (W.Job(61, 6, 1000, 4003, 300, 10**6), 24),          # ragged last tile, gaps 2 and 4
    (W.Job(61, 6, 1000, 4003, 300, 10**6), 100),
    (W.Job(97, 1, 7, 1501, 250, 3 * 10**6), 40),         # d = 1: every m, gap 1
    (W.Job(131, 210, 10**6, 20011, 700, 5 * 10**6), 52),  # gaps up to 10
    (W.Job(97, 30030, 1, 90000, 400, 2 * 10**6), 30),     # gaps up to 22: tiles without the pass
    (W.Job(503, 210, 10**6, 3000, 7000, 10**7), 30),
], ids=["d6_24w", "d6_100w", "d1_40w", "d210_52w", "d30030_30w", "p503_30w"])
def test_small_branch_hit_rows(job, mult):
    """Thresholds of 24 w and more run the small branch's hit-row pass (offsets stepped over the
    tile's rows, then each lane's hit rows marked): every row equals the oracle's."""
    w = 2 * job.sl
    tune = cs.Tune(thr=mult * w, large_mode=cs.LARGE_THREE_GAP)
    assert cs.plan(job, tune).thr == mult * w
    _say("hit rows", job, mult)
    got_b, got_c, diag, _ = _run(job, tune)
    want_b, want_c = _oracle(job)
    _assert_same(job, got_b, got_c, want_b, want_c)
    assert diag.error_flags == 0 and diag.small_marks > 0


@pytest.mark.parametrize("thr", [2**31 - 1, 2**32], ids=["thr_below_2^31", "thr_2^32"])
def test_small_branch_primes_above_2_31(thr):
    """Small-branch primes just above 2^31 (a threshold set at or beyond 2^31 sends them through
    the 64-bit residue path of the small branch, one below it through the large branch): the marks
    of every row equal the oracle's."""
    lo, hi = 2**31, 2**31 + 2**22
    job = W.Job(61, 6, 1000, 4000, 3000, hi)
    tune = cs.Tune(thr=thr, large_mode=cs.LARGE_THREE_GAP)
    _say("small branch above 2^31", thr)
    lay, bitmap, counts, ws = cs.binding.alloc_outputs(job, tune)
    bitmap.zero_()
    counts.zero_()
    cs.prepare(job, ws, tune)
    cs.sieve_range(job, lo, hi, bitmap, counts, ws, tune)
    torch.cuda.synchronize()
    m_all = coracle.rows(job.d, job.m_start, job.m_inc)
    want_b, want_c = coracle.sieve_rows(job.P, job.d, job.sl, m_all, lo, hi, mode=coracle.CACHED)
    assert want_c.sum() > 100
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), want_c)
    assert np.array_equal(bitmap.cpu().numpy().view(np.uint32), want_b)


def test_window_hits_503_from_large_branch(paper_values):
    """Section 3.2's statistics for N = 503#/210, X = 1e5, reproduced by the large branch's own
    count of Eq. 3 solutions (one m, so each hit is one prime dividing the interval)."""
    w = paper_values["window_hits_503"]
    job = W.Job(w["P"], w["d"], w["m"], 1, w["sl"], 10**9)
    tune = cs.Tune(thr=2 * w["sl"])
    lay, bitmap, counts, _ = cs.binding.alloc_outputs(job, tune)
    ws_bytes = max(cs.plan(job, cs.Tune(thr=2 * w["sl"])).ws_bytes,
                   cs.plan(job, cs.Tune(thr=4 * w["sl"] + 1, large_mode=cs.LARGE_THREE_GAP)).ws_bytes)
    ws = torch.empty((ws_bytes,), dtype=torch.uint8, device="cuda")    # fits both tunings
    for mode in (cs.LARGE_G, cs.LARGE_THREE_GAP):
        tune.large_mode = mode
        tune.thr = 2 * w["sl"] if mode == cs.LARGE_G else 4 * w["sl"] + 1
        cs.prepare(job, ws, tune)
        for rg in w["ranges"][1:]:
            if rg["lo"] <= tune.thr:
                continue
            before = cs.diag_read(ws).large_raw_hits
            cs.sieve_range(job, rg["lo"], rg["hi"], bitmap, counts, ws, tune)
            got = cs.diag_read(ws).large_raw_hits - before
            assert got == rg["hit"], (mode, rg)


def test_repeat_is_deterministic():
    job = W.Job(307, 30, 10**5, 20000, 3000, 2 * 10**7)
    a = _run(job)
    b = _run(job)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_zero_rows():
    job = W.Job(11, 2, 4, 1, 5, 100)
    bitmap, counts, ws = cs.sieve(job)
    torch.cuda.synchronize()
    assert bitmap.numel() == 0 and counts.numel() == 0


def test_large_kernel_time_is_reported():
    """cs_diag.large_kernel_ms: the last large-branch launch on the workspace, timed by HIP events."""
    job = W.MEDIUM
    lay, bitmap, counts, ws = cs.binding.alloc_outputs(job)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cs.sieve_into(job, bitmap, counts, ws)
    e0.record(s)
    cs.sieve_into(job, bitmap, counts, ws)
    e1.record(s)
    d = cs.diag_read(ws)
    assert 0.0 < d.large_kernel_ms <= e0.elapsed_time(e1)


def _random_cases(seed, n):
    """Seeded random small jobs and tunings (P <= 101, d a product of P's smallest primes, m_start
    and m_inc from 1, limits to 1e6, every enumeration, scatter and threshold kind); invalid
    combinations (e.g. d not squarefree) are dropped by the planner."""
    import random
    rng = random.Random(seed)
    primes = [int(p) for p in coracle.primes_range(2, 101)]
    out = []
    while len(out) < n:
        P = rng.choice(primes)
        small = [q for q in primes if q <= P]
        d = 1
        for q in small[:6]:
            if rng.random() < 0.4:
                d *= q
        job = W.Job(P, d, rng.choice([1, 2, 3, rng.randrange(1, 10**6)]), rng.choice([1, 2, 3, rng.randrange(1, 400)]),
                    rng.randrange(1, 600), rng.choice([rng.randrange(2, 2000), rng.randrange(2, 10**6)]))
        tune = cs.Tune(large_mode=rng.choice([cs.LARGE_G, cs.LARGE_THREE_GAP]),
                       thr=rng.choice([0, 0, 1, rng.randrange(1, 5000), 10**9]),
                       scatter=rng.choice([cs.SCATTER_AUTO, cs.SCATTER_ATOMIC, cs.SCATTER_BYTES, cs.SCATTER_LIST]))
        try:
            cs.plan(job, tune)
        except cs.CsError:
            continue
        out.append((job, tune))
    return out


@pytest.mark.parametrize("seed", [11, 12])
def test_random_jobs_match_oracle(seed):
    """60 seeded random jobs per seed: bitmap and counts equal the oracle's (bignum residues)."""
    for job, tune in _random_cases(seed, 60):
        _say("random", seed, job, tune.large_mode, tune.thr, tune.scatter)
        got_b, got_c, _, _ = _run(job, tune)
        want_b, want_c = _oracle(job, mode=coracle.DIRECT)
        _assert_same(job, got_b.reshape(want_b.shape), got_c, want_b, want_c)

"""Pins of the CPU oracle against facts that do not come from the oracle itself:
brute-force trial division on tiny K, numbers printed in the paper, closed forms and the
invariants of the deficient-primorial construction (Section 2, "Primorials")."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import coracle, plain


# ----------------------------------------------------------------------------------------
# Brute force: factor every N = m*K + X by trial division, independent of any sieve.
# ----------------------------------------------------------------------------------------
def _is_prime(n):
    if n < 2:
        return False
    q = 2
    while q * q <= n:
        if n % q == 0:
            return False
        q += 1
    return True


def _prime_factors_upto(n, limit):
    """Distinct primes q <= limit with q | n (trial division up to min(limit, n))."""
    out = []
    q = 2
    while q <= limit and q <= n:
        if n % q == 0 and _is_prime(q):
            out.append(q)
        q += 1
    return out


def brute_force(job):
    P, d, m_start, m_inc, sl, limit = job.as_tuple()
    K = 1
    for q in range(2, P + 1):
        if _is_prime(q):
            K *= q
    assert K % d == 0
    K //= d
    ms = [m for m in range(m_start, m_start + m_inc) if math.gcd(m, d) == 1]
    xs = [X for X in range(-sl, sl + 1) if math.gcd(X, K) == 1]
    bits = np.zeros((len(ms), len(xs)), dtype=np.uint8)
    counts = np.zeros(len(ms), dtype=np.uint32)
    for i, m in enumerate(ms):
        for c, X in enumerate(xs):
            f = _prime_factors_upto(m * K + X, limit)
            bits[i, c] = 1 if f else 0
            counts[i] += len(f)
    return xs, ms, bits, counts


def _tiny_cases():
    cases = [W.Job(11, d, 3, 40, 60, 3000) for d in (1, 2, 6, 30, 210)]
    cases += [W.Job(11, 210, 1, 30, 10, 200), W.Job(13, 2, 1, 25, 200, 997)]
    cases += W.tiny_jobs(seed=7, n=25)
    return cases


@pytest.mark.parametrize("job", _tiny_cases(), ids=lambda j: "P%d_d%d_m%d+%d_sl%d_L%d" % j.as_tuple())
def test_oracle_matches_trial_division(job):
    xs, ms, bits, counts = brute_force(job)
    assert list(coracle.columns(job.P, job.d, job.sl)) == xs
    assert list(coracle.rows(job.d, job.m_start, job.m_inc)) == ms
    for mode in (coracle.DIRECT, coracle.CACHED):
        b, c = coracle.sieve_job(job, mode=mode)
        assert np.array_equal(plain.unpack(b, len(xs)), bits)
        assert np.array_equal(c, counts)
    pb, pc = plain.sieve(job)
    assert np.array_equal(pb, bits) and np.array_equal(pc, counts)


def test_witness_divides(paper_values):
    """Every marked bit carries a prime that divides m*K + X (checked with Python bignums)."""
    job = W.SMALL
    K = plain.K_of(job.P, job.d)
    xs = coracle.columns(job.P, job.d, job.sl)
    ms = coracle.rows(job.d, job.m_start, job.m_inc)
    bits, counts, wit = coracle.sieve_job(job, mode=coracle.DIRECT, witness=True)
    u = plain.unpack(bits, len(xs))
    assert np.array_equal(u != 0, wit != 0)
    rng = np.random.default_rng(3)
    rr, cc = np.nonzero(wit)
    pick = rng.choice(len(rr), size=2000, replace=False)
    for i in pick:
        m, X, p = int(ms[rr[i]]), int(xs[cc[i]]), int(wit[rr[i], cc[i]])
        assert (m * K + X) % p == 0
        assert all((m * K + X) % q for q in plain.primes_upto(p - 1)[:50] if q < p)
    # unmarked bits have no factor among the first primes that can divide them
    ur, uc = np.nonzero(u == 0)
    for i in rng.choice(len(ur), size=min(300, len(ur)), replace=False):
        n = int(ms[ur[i]]) * K + int(xs[uc[i]])
        assert all(n % q for q in plain.primes_upto(2000))
    # counts are at least the number of marked bits
    assert np.all(counts >= u.sum(axis=1))


# ----------------------------------------------------------------------------------------
# Numbers printed in the paper.
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("x", [10**4, 10**5, 200001, 10**6, 10**8])
def test_prime_counts(paper_values, x):
    n, _ = coracle.prime_stats(2, x)
    assert n == paper_values["prime_counts"][str(x)]


def _digits_ok(value, printed):
    """value agrees with the printed decimal to its last digit (rounded or truncated)."""
    dec = len(printed.split(".")[1])
    unit = 10.0 ** -dec
    return abs(value - float(printed)) <= unit


@pytest.mark.parametrize("x", [10**4, 10**5, 10**6, 10**8])
def test_mertens_experimental(paper_values, x):
    _, s = coracle.prime_stats(2, x)
    assert _digits_ok(math.exp(s), paper_values["mertens_experimental"][str(x)])


@pytest.mark.slow
@pytest.mark.parametrize("x", [4 * 10**9, 10**10])
def test_prime_counts_large(paper_values, x):
    n, s = coracle.prime_stats(2, x)
    assert n == paper_values["prime_counts"][str(x)]
    assert _digits_ok(math.exp(s), paper_values["mertens_experimental"][str(x)])


def test_pi_1e9(paper_values):
    n, _ = coracle.prime_stats(2, 10**9)
    assert n == paper_values["prime_counts"]["1000000000"]


def test_window_hits_503(paper_values):
    """Section 3.2: how many primes of each range divide a number of [N - X, N + X]."""
    w = paper_values["window_hits_503"]
    for rg in w["ranges"]:
        n, _ = coracle.prime_stats(rg["lo"], rg["hi"])
        assert n == rg["primes"]
        hit = coracle.window_hit_primes(w["P"], w["d"], w["m"], w["sl"], rg["lo"], rg["hi"])
        assert hit == rg["hit"], rg


def test_coprime_m_count(paper_values):
    c = paper_values["coprime_m_count"]
    assert len(coracle.rows(c["d"], 1, c["M"])) == c["M_c"]
    assert len(plain.rows(c["d"], 1, c["M"])) == c["M_c"]


# ----------------------------------------------------------------------------------------
# Invariants of the primorial construction (Section 2, "Primorials").
# ----------------------------------------------------------------------------------------
@pytest.mark.parametrize("P", [13, 31, 211])
def test_d1_small_offsets_are_not_columns(P):
    xs = set(int(x) for x in coracle.columns(P, 1, 3 * P))
    for X in range(2, P + 1):
        assert X not in xs and -X not in xs
    assert 1 in xs and -1 in xs


@pytest.mark.parametrize("P", [31, 211])
def test_d2_parity_and_powers_of_two(P):
    sl = 4 * P
    xs = [int(x) for x in coracle.columns(P, 2, sl)]
    even = sorted(x for x in xs if x % 2 == 0 and abs(x) <= 2 * P)
    pw = sorted({s * 2**a for a in range(1, 20) for s in (1, -1) if 2**a <= 2 * P})
    assert even == pw
    ms = coracle.rows(2, 1, 40)
    bits, _ = coracle.sieve_rows(P, 2, sl, ms, 2, 2)          # the prime 2 alone
    u = plain.unpack(bits, len(xs))
    odd = np.array([x % 2 != 0 for x in xs])
    assert np.all(u[:, odd] == 1) and np.all(u[:, ~odd] == 0)


def test_columns_match_between_oracles():
    for P, d, sl in [(211, 210, 4000), (503, 30, 500), (97, 1, 800)]:
        assert list(coracle.columns(P, d, sl)) == plain.columns(P, d, sl)


@pytest.mark.slow
def test_record_gap_953_row(paper_values):
    """The prime 100054841*953#/210 - 9670 has no factor up to 1e10: its bit stays clear.
    The whole row is also internally consistent (witness divides)."""
    g = paper_values["record_gaps"]["gaps"][0]
    job = W.PAPER_SCALE
    xs = [int(x) for x in coracle.columns(job.P, job.d, job.sl)]
    c = xs.index(g["x_prev"])
    bits, counts = coracle.sieve_rows(job.P, job.d, job.sl, [g["m"]], 2, job.limit, mode=coracle.CACHED)
    u = plain.unpack(bits, len(xs))
    assert u[0, c] == 0
    assert g["x_prev"] + g["gap"] > job.sl     # the next prime lies beyond the window
    assert u[0].sum() < len(xs) and counts[0] >= u[0].sum()


def test_record_gap_1019_row(paper_values):
    g = paper_values["record_gaps"]["gaps"][1]
    sl = 20000
    xs = [int(x) for x in coracle.columns(g["P"], g["d"], sl)]
    bits, _ = coracle.sieve_rows(g["P"], g["d"], sl, [g["m"]], 2, 10**8, mode=coracle.DIRECT)
    u = plain.unpack(bits, len(xs))
    assert u[0, xs.index(g["x_prev"])] == 0
    assert u[0, xs.index(g["x_prev"] + g["gap"])] == 0


def test_direct_and_cached_agree_medium_rows():
    """The Eq. 1 identity: r from the bignum and r from (m mod p)(K mod p) give the same rows."""
    job = W.MEDIUM
    ms = coracle.rows(job.d, job.m_start, job.m_inc)[[0, 17, 1000, -1]]
    a = coracle.sieve_rows(job.P, job.d, job.sl, ms, 2, 3 * 10**6, mode=coracle.DIRECT)
    b = coracle.sieve_rows(job.P, job.d, job.sl, ms, 2, 3 * 10**6, mode=coracle.CACHED)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_prime_range_split_is_additive():
    """Sieving [2, L] equals OR / sum of sieving [2, a] and [a+1, L] (used by range calls)."""
    job = W.SMALL
    ms = coracle.rows(job.d, job.m_start, job.m_inc)
    full = coracle.sieve_rows(job.P, job.d, job.sl, ms, 2, job.limit)
    lo = coracle.sieve_rows(job.P, job.d, job.sl, ms, 2, 5003)
    hi = coracle.sieve_rows(job.P, job.d, job.sl, ms, 5004, job.limit)
    assert np.array_equal(full[0], lo[0] | hi[0])
    assert np.array_equal(full[1], lo[1] + hi[1])


def _is_prime_mr(n: int) -> bool:
    """Deterministic Miller-Rabin below 3.4e14 (bases 2..17), for pinning the oracle's primes."""
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 11, 13, 17):
        if n % q == 0:
            return n == q
    dd, s = n - 1, 0
    while dd % 2 == 0:
        dd //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17):
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


def test_oracle_near_2_42():
    """At the largest primes the library takes (just below 2^42): the oracle's primes are the
    primes, its N mod p equals Python's big-integer N mod p, its bignum and cached residues
    (Eq. 1) give the same rows over a window of primes, and every mark it makes there has a
    witness prime that divides N + X."""
    P, d, sl = 61, 6, 131000
    K = plain.K_of(P, d)
    lo, hi = 2**42 - 2**20, 2**42 - 1
    ps = coracle.primes_range(lo, hi)
    sample = [int(p) for p in ps[:: max(1, len(ps) // 400)]]
    assert all(_is_prime_mr(p) for p in sample)
    gaps = [n for n in range(hi - 3000, hi + 1) if _is_prime_mr(n)]
    assert [int(p) for p in ps if p > hi - 3000] == gaps          # no prime missed at the top
    m = 10**6 + 1
    got = coracle.n_mod(P, d, m, ps[:3000])
    assert [int(v) for v in got] == [(m * K) % int(p) for p in ps[:3000]]
    ms = coracle.rows(d, 10**6, 48000)
    a_b, a_c = coracle.sieve_rows(P, d, sl, ms, lo, hi, mode=coracle.DIRECT)
    b_b, b_c = coracle.sieve_rows(P, d, sl, ms, lo, hi, mode=coracle.CACHED)
    assert np.array_equal(a_b, b_b) and np.array_equal(a_c, b_c)
    xs = [int(x) for x in coracle.columns(P, d, sl)]
    hit = ms[np.nonzero(a_c)[0]]                       # witnesses only for the rows with marks
    h_b, h_c, wit = coracle.sieve_rows(P, d, sl, hit, lo, hi, mode=coracle.DIRECT, witness=True)
    marked = np.argwhere(plain.unpack(h_b, len(xs)))
    assert len(marked) >= 3 and len(marked) == int(a_c.sum()) == int(h_c.sum())
    for r, c in marked:
        w = int(wit[r, c])
        assert lo <= w <= hi and (int(hit[r]) * K + xs[c]) % w == 0

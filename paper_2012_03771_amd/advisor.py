"""Parameter advisor (Section 4 of the paper): how far to sieve and how wide an interval to sieve.

* Eq. 6 (Mertens' third theorem): the fraction of integers with no prime factor <= P_limit is
  about 1 / (log(P_limit) e^gamma).
* Eq. 7: near N, after that sieve, finding a prime takes about
  E(N, P_limit) = log(N) / (log(P_limit) e^gamma) probable-prime tests.
* Sieve limit: sieving one more range of primes (P1, P2] saves every interval about
  2 (E(N, P1) - E(N, P2)) tests (one search on each side of N); keep sieving while the tests
  saved per second of sieving exceed the measured probable-prime test rate.
* Interval: X between 6 log N and 10 log N; warn when a test sieve of a few m finds the
  surrounding primes beyond X more than 0.5% of the time.

The formulas are host arithmetic; the rates come from timing the library's own kernels (the
range sieve and the probable-prime test) on the GPU.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

EULER_GAMMA = 0.5772156649015329


def mertens_fraction(p_limit: float) -> float:
    """Eq. 6: about the fraction of integers with no prime factor <= p_limit."""
    return 1.0 / (math.log(p_limit) * math.exp(EULER_GAMMA))


def expected_tests(log_n: float, p_limit: float) -> float:
    """Eq. 7: probable-prime tests expected to find one prime near N (log_n = natural log of N)
    among numbers with no prime factor <= p_limit."""
    return log_n / (math.log(p_limit) * math.exp(EULER_GAMMA))


def log_n_of(job) -> float:
    """Natural log of N = m_start * P#/d."""
    from . import binding as B
    P, d, m_start, _, _, _ = B.job_tuple(job)
    s = math.log(m_start) - math.log(d)
    for q in _primes_upto(P):
        s += math.log(q)
    return s


def interval_range(log_n: float) -> tuple[int, int]:
    """Section 4.2: X (= sl) between 6 log N and 10 log N."""
    return int(math.ceil(6 * log_n)), int(math.floor(10 * log_n))


def _primes_upto(n: int) -> list[int]:
    if n < 2:
        return []
    sieve = bytearray([1]) * (n + 1)
    sieve[0] = sieve[1] = 0
    for i in range(2, int(n ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = bytearray(len(sieve[i * i::i]))
    return [i for i in range(n + 1) if sieve[i]]


@dataclass
class RangeStep:
    p_lo: int
    p_hi: int
    ms: float                  # time of cs_sieve_range over (p_lo, p_hi] for the whole job
    tests_saved: float         # over all rows: 2 n_m (E(N, p_lo) - E(N, p_hi))
    saved_per_s: float


@dataclass
class LimitAdvice:
    limit: int                 # advised sieve limit (the end of the last range worth sieving)
    prp_tests_per_s: float
    steps: list = field(default_factory=list)


def prp_rate(job, n_tests: int = 1 << 15, seed: int = 0, stream=None) -> float:
    """Measured strong-test rate (tests/s) on random odd numbers of N's size (cs_prp_numbers)."""
    import numpy as np
    import torch
    from . import binding as B
    bits = int(log_n_of(job) / math.log(2)) + 1
    n_limbs = (bits + 31) // 32
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 2**32, size=(n_tests, n_limbs), dtype=np.uint64).astype(np.uint32)
    top = bits - 32 * (n_limbs - 1)
    a[:, -1] = (a[:, -1] & np.uint32((1 << top) - 1 if top < 32 else 0xffffffff)) | np.uint32(1 << (top - 1))
    a[:, 0] |= np.uint32(1)
    t = torch.from_numpy(a.view(np.int32)).cuda()
    s = stream or torch.cuda.current_stream()
    B.prp_numbers(t, s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    B.prp_numbers(t, s)
    e1.record(s)
    e1.synchronize()
    return n_tests / (e0.elapsed_time(e1) / 1e3)


def advise_sieve_limit(job, prp_tests_per_s: float | None = None, first: int | None = None,
                       factor: float = 4.0, tune=None, stream=None) -> LimitAdvice:
    """Sieves the job in geometrically growing prime ranges up to job.limit (cs_prepare, then
    cs_sieve_range per range, each timed with HIP events) and returns the end of the last range
    whose saved tests per second of sieving still exceed the probable-prime test rate."""
    import torch
    from . import binding as B
    lay, bitmap, counts, ws = B.alloc_outputs(job, tune)
    s = stream or torch.cuda.current_stream()
    rate = prp_tests_per_s if prp_tests_per_s is not None else prp_rate(job, stream=s)
    log_n = log_n_of(job)
    limit = B.job_tuple(job)[5]
    bitmap.zero_()
    counts.zero_()
    B.prepare(job, ws, tune, s)
    lo = 1
    hi = first if first is not None else max(2, min(limit, 1000))
    steps = []
    advised = hi
    while True:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        B.sieve_range(job, lo + 1, hi, bitmap, counts, ws, tune, s)
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        saved = 2.0 * lay.n_m * (expected_tests(log_n, max(lo, 2)) - expected_tests(log_n, hi)) if lo > 1 else 0.0
        per_s = saved / max(ms / 1e3, 1e-9)
        steps.append(RangeStep(lo, hi, ms, saved, per_s))
        if lo == 1 or per_s >= rate:
            advised = hi
        if hi >= limit:
            break
        lo, hi = hi, min(limit, int(hi * factor))
    del bitmap, counts, ws
    return LimitAdvice(advised, rate, steps)


@dataclass
class IntervalAdvice:
    sl: int
    recommended: tuple
    rows: int
    beyond: int                # rows whose previous or next probable prime lies beyond sl
    fraction: float
    warn: bool


def check_interval(job, rows: int = 256, stream=None) -> IntervalAdvice:
    """Test sieve of the first `rows` rows (cs_sieve on a job of that many m), then the surrounding
    probable primes (cs_surround); warns if more than 0.5% of them lie beyond sl."""
    import numpy as np
    import torch
    from . import binding as B
    P, d, m_start, m_inc, sl, limit = B.job_tuple(job)
    small = (P, d, m_start, min(m_inc, rows * d // _phi(d) + d), sl, limit)   # about `rows` coprime m
    bm, cn, ws = B.sieve(small, stream=stream)
    ms = B.rows(small)[:rows]
    out, _ = B.surround(small, bm[:len(ms)].contiguous(), torch.from_numpy(ms.astype(np.int64)).cuda(), stream=stream)
    o = out.cpu().numpy()
    beyond = int(((o[:, 0] == 0) | (o[:, 1] == 0)).sum())
    frac = beyond / max(1, len(ms))
    return IntervalAdvice(sl, interval_range(log_n_of(job)), len(ms), beyond, frac, frac > 0.005)


def _phi(d: int) -> int:
    r, n, q = d, d, 2
    while q * q <= n:
        if n % q == 0:
            while n % q == 0:
                n //= q
            r -= r // q
        q += 1
    if n > 1:
        r -= r // n
    return r

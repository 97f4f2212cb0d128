"""Seeded synthetic sieve jobs shared by the tests, the benchmark and the oracle scripts.

A job is the parameter set of the Combined Sieve problem statement (Section 3 of the paper):
K = P#/d, rows m in [m_start, m_start + m_inc) with gcd(m, d) = 1, offsets X in [-sl, sl]
with gcd(X, K) = 1, and every prime p <= limit is sieved.  The method has no data set: its
inputs are these integers, so every workload here is synthetic by construction.

This module holds only the job recipes.  It performs none of the sieve's arithmetic and
imports neither the oracle nor the HIP package.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np


@dataclass(frozen=True)
class Job:
    P: int          # primorial bound: K = P#/d
    d: int          # squarefree divisor of P#
    m_start: int    # first multiplier
    m_inc: int      # number of multipliers scanned (only those coprime to d become rows)
    sl: int         # half width of each interval: X in [-sl, sl]
    limit: int      # sieve limit: primes p <= limit are sieved

    def as_tuple(self):
        return (self.P, self.d, self.m_start, self.m_inc, self.sl, self.limit)

    def to_dict(self):
        return asdict(self)


# Single-job workloads at the sizes of the paper's experiments (Section 3 and Appendix):
# a small primorial that the oracle finishes in seconds, a mid-size one that exercises both
# prime branches with 32-bit primes, and a paper-scale one (953#/210, the primorial of the
# merit-38.048 record gap of Section 1.1) with primes up to 1e10.
SMALL = Job(211, 210, 1, 1000, 4000, 10**6)
MEDIUM = Job(503, 210, 10**6, 10**4, 7000, 10**8)
PAPER_SCALE = Job(953, 210, 10**8, 10**6, 20000, 10**10)

SINGLE_JOBS = {"small_211": SMALL, "medium_503": MEDIUM, "paper_953": PAPER_SCALE}

# Record gaps of Section 1.1: (P, d, m, X of the prime that starts the gap, gap length).
RECORD_GAPS = [
    (953, 210, 100054841, -9670, 35308),
    (1019, 210, 164065661, -18566, 36702),
]


def _small_primes(lo: int, hi: int):
    """Primes in [lo, hi] by trial division (input recipe only; hi is at most a few thousand)."""
    out = []
    for n in range(max(lo, 2), hi + 1):
        if all(n % q for q in range(2, int(n ** 0.5) + 1)):
            out.append(n)
    return out


def ln_primorial_over_d(P: int, d: int) -> float:
    return sum(math.log(q) for q in _small_primes(2, P)) - math.log(d)


def interval_half_width(m_start: int, P: int, d: int) -> int:
    """sl = round(40 * ln N) with N = m_start * P#/d (natural log, as the paper's merit uses)."""
    return int(math.floor(40.0 * (math.log(m_start) + ln_primorial_over_d(P, d)) + 0.5))


BATCH_P_CHOICES = _small_primes(307, 1019)      # 109 primes
BATCH_D_CHOICES = (1, 2, 6, 30, 210)


def random_job(rng: np.random.Generator) -> Job:
    """One job of the mixed batch: P uniform over primes in [307, 1019], d uniform over
    {1, 2, 6, 30, 210}, m_inc log-uniform in [1e3, 1e5], limit log-uniform in [1e7, 1e9],
    m_start log-uniform in [1, 1e9], sl = round(40 ln N)."""
    P = int(BATCH_P_CHOICES[int(rng.integers(0, len(BATCH_P_CHOICES)))])
    d = int(BATCH_D_CHOICES[int(rng.integers(0, len(BATCH_D_CHOICES)))])
    m_inc = int(round(10 ** rng.uniform(3.0, 5.0)))
    limit = int(round(10 ** rng.uniform(7.0, 9.0)))
    m_start = max(1, int(round(10 ** rng.uniform(0.0, 9.0))))
    sl = interval_half_width(m_start, P, d)
    return Job(P, d, m_start, m_inc, sl, limit)


def batch_jobs(n: int = 64, seed: int = 0):
    rng = np.random.default_rng(seed)
    return [random_job(rng) for _ in range(n)]


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 1):
    """Arrival times (s) of a Poisson stream and the jobs that arrive, both seeded."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    times = np.cumsum(gaps) - gaps[0]
    jobs = [random_job(rng) for _ in range(n)]
    return times.tolist(), jobs


def tiny_jobs(seed: int, n: int, max_P: int = 31):
    """Small jobs for brute-force cross checks: K = P#/d with P <= max_P, short intervals."""
    rng = np.random.default_rng(seed)
    ps = _small_primes(2, max_P)
    out = []
    for _ in range(n):
        P = int(ps[int(rng.integers(1, len(ps)))])
        dprimes = [q for q in ps if q <= P and rng.random() < 0.4]
        d = 1
        for q in dprimes:
            d *= q
        m_start = int(rng.integers(1, 500))
        m_inc = int(rng.integers(1, 60))
        sl = int(rng.integers(1, 300))
        limit = int(rng.integers(2, 3000))
        K = 1
        for q in ps:
            if q <= P:
                K *= q
        K //= d
        if m_start * K < 2:
            m_start = 2
        if sl >= m_start * K:            # keep every N = m*K + X positive
            sl = max(1, m_start * K - 1)
        out.append(Job(P, d, m_start, m_inc, sl, limit))
    return out


def sample_rows(n_rows: int, k: int, seed: int, must=()):
    """k row indices: the first, the last, the given ones, and seeded picks."""
    rng = np.random.default_rng(seed)
    rows = {0, n_rows - 1, *[r for r in must if 0 <= r < n_rows]}
    while len(rows) < min(k, n_rows):
        rows.add(int(rng.integers(0, n_rows)))
    return sorted(rows)

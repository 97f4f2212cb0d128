"""Surrounding-prime oracle (test infrastructure only).

After the sieve, the search for a large gap around N = m*K tests the unmarked numbers N + X for
primality, walking away from N on each side, until the nearest probable prime below and above N
is found (Section 2, "Larger Gaps" and "Sieving"; Section 2.2 on probabilistic tests).  The gap is
their distance and its merit is the gap over log of the lower prime (Section 1).

The probable-prime test here is the strong test to base 2 (the first half of BPSW, the test the
paper's search runs through GMP): write n - 1 = 2^s * t with t odd; n passes iff 2^t = 1 (mod n)
or 2^(2^r * t) = -1 (mod n) for some 0 <= r < s.  Every prime passes; odd composites that pass
are the strong pseudoprimes to base 2.  Python's built-in modular power is the one library
primitive used.
"""
from __future__ import annotations

import math
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import plain


def sprp2(n: int) -> bool:
    """Strong probable-prime test to base 2 (definition above)."""
    if n < 2:
        return False
    if n == 2:
        return True
    if n % 2 == 0:
        return False
    t, s = n - 1, 0
    while t % 2 == 0:
        t //= 2
        s += 1
    y = pow(2, t, n)
    if y == 1 or y == n - 1:
        return True
    for _ in range(s - 1):
        y = y * y % n
        if y == n - 1:
            return True
    return False


def candidates(P: int, d: int, sl: int, bits_row=None):
    """Both sides' candidate offsets in test order: X = -1, -2, ... and X = 1, 2, ... restricted to
    the columns (gcd(X, K) = 1) and, when a sieved row is given (one uint8 per column, 1 =
    marked), to its unmarked columns."""
    cols = plain.columns(P, d, sl)
    if bits_row is not None:
        keep = [X for X, b in zip(cols, bits_row) if not b]
    else:
        keep = cols
    below = [X for X in reversed(keep) if X < 0]
    above = [X for X in keep if X > 0]
    return below, above


def _first_prp(N: int, xs, trial_product: int) -> tuple[int, int]:
    for i, X in enumerate(xs):
        if trial_product > 1 and math.gcd(N + X, trial_product) > 1:
            continue                       # a prime below the trial bound divides it (N + X is larger)
        if sprp2(N + X):
            return X, i + 1
    return 0, len(xs)


def surround(P: int, d: int, m: int, sl: int, bits_row=None, trial: int = 0) -> tuple[int, int, int, int]:
    """(prev, next, tests_prev, tests_next) for N = m * P#/d.

    prev = the largest X < 0 with N + X a probable prime, next = the smallest X > 0 with N + X a
    probable prime, searched only within [-sl, sl]; 0 means none there.  tests_* counts the
    candidates examined on that side up to and including the one found (all of them if none).
    trial > 0 skips candidates with a prime factor <= trial (by one gcd with their product); it
    changes no prev/next when N - sl exceeds trial, only the work."""
    K = plain.K_of(P, d)
    N = m * K
    tp_ = plain.primorial(trial) if trial > 0 else 1
    below, above = candidates(P, d, sl, bits_row)
    prev, tp = _first_prp(N, below, tp_)
    nxt, tn = _first_prp(N, above, tp_)
    return prev, nxt, tp, tn


def _surround_args(a):
    return surround(*a)


def surround_rows(P: int, d: int, ms, sl: int, bits=None, workers: int = 8, trial: int = 0):
    """surround() for many rows, in parallel processes; bits = unpacked sieve rows or None."""
    args = [(P, d, int(m), sl, None if bits is None else bits[i], trial) for i, m in enumerate(ms)]
    if workers <= 1 or len(args) == 1:
        return [surround(*a) for a in args]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_surround_args, args, chunksize=max(1, len(args) // (4 * workers))))


def merit(P: int, d: int, m: int, prev: int, nxt: int) -> float:
    """gap / log(lower prime) (Section 1)."""
    N = m * plain.K_of(P, d) + prev
    return (nxt - prev) / (math.log2(N) * math.log(2.0))


def interior_composite(P: int, d: int, m: int, xs, workers: int = 8) -> bool:
    """True iff every N + X for X in xs fails the test (checked in parallel processes)."""
    N = m * plain.K_of(P, d)
    ns = [N + int(X) for X in xs]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return not any(ex.map(sprp2, ns, chunksize=max(1, len(ns) // (8 * workers))))


def limbs(n: int, n_limbs: int) -> np.ndarray:
    """n as little-endian 32-bit limbs."""
    return np.array([(n >> (32 * i)) & 0xffffffff for i in range(n_limbs)], dtype=np.uint32)

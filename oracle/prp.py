"""Surrounding-prime oracle (test infrastructure only).

After the sieve, the search for a large gap around N = m*K tests the unmarked numbers N + X for
primality, walking away from N on each side, until the nearest probable prime below and above N
is found (Section 2, "Larger Gaps" and "Sieving"; Section 2.2 on probabilistic tests).  The gap is
their distance and its merit is the gap over log of the lower prime (Section 1).

The paper's search tests with GMP's probable-prime routine, a BPSW test (Section 2.2): the
strong test to base 2 and a strong Lucas test.

Strong test to base 2: write n - 1 = 2^s * t with t odd; n passes iff 2^t = 1 (mod n) or
2^(2^r * t) = -1 (mod n) for some 0 <= r < s.  Every prime passes; odd composites that pass are
the strong pseudoprimes to base 2.

Strong Lucas test (Baillie and Wagstaff, 1980, with Selfridge's parameters): for odd n > 1 not a
perfect square, D is the first of 5, -7, 9, -11, 13, ... with Jacobi symbol (D/n) = -1, P = 1,
Q = (1 - D)/4.  The Lucas sequences are U_0 = 0, U_1 = 1, V_0 = 2, V_1 = P and
W_{k+1} = P W_k - Q W_{k-1}.  Write n + 1 = 2^s * d with d odd; n passes iff U_d = 0 (mod n) or
V_(2^r d) = 0 (mod n) for some 0 <= r < s.  Every prime not dividing 2QD passes.  A D with
(D/n) = 0 and |D| != n shows a factor of n.

BPSW: n passes both.  No composite is known to pass.  Python's built-in modular power is the one
library primitive used.
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


def jacobi(a: int, n: int) -> int:
    """Jacobi symbol (a/n) for odd n > 0: the product of the Legendre symbols over the prime
    factors of n, computed by quadratic reciprocity and the rules for (2/n) and (-1/n)."""
    assert n > 0 and n % 2 == 1
    a %= n
    t = 1
    while a != 0:
        while a % 2 == 0:
            a //= 2
            if n % 8 in (3, 5):
                t = -t
        a, n = n, a
        if a % 4 == 3 and n % 4 == 3:
            t = -t
        a %= n
    return t if n == 1 else 0


def selfridge(n: int):
    """(D, P, Q) for the strong Lucas test of odd n > 1 that is not a perfect square; None when a
    D with (D/n) = 0 and |D| != n shows that n is composite."""
    D = 5
    while True:
        j = jacobi(D, n)
        if j == -1:
            return D, 1, (1 - D) // 4
        if j == 0 and abs(D) != n:
            return None
        D = -(D + 2) if D > 0 else -D + 2


def lucas_uv(P: int, Q: int, k: int, n: int) -> tuple[int, int, int]:
    """(U_k, V_k, Q^k) mod n by the doubling formulas U_2k = U_k V_k, V_2k = V_k^2 - 2 Q^k and the
    step U_(k+1) = (P U_k + V_k)/2, V_(k+1) = (D U_k + P V_k)/2 (D = P^2 - 4Q), over the bits of k
    from the top; n odd, so halving mod n is exact."""
    D = P * P - 4 * Q
    inv2 = (n + 1) // 2
    if k == 0:
        return 0, 2 % n, 1 % n
    U, V, Qk = 1 % n, P % n, Q % n
    for bit in bin(k)[3:]:
        U, V, Qk = U * V % n, (V * V - 2 * Qk) % n, Qk * Qk % n
        if bit == "1":
            U, V = (P * U + V) * inv2 % n, (D * U + P * V) * inv2 % n
            Qk = Qk * Q % n
    return U, V, Qk


def strong_lucas(n: int) -> bool:
    """Strong Lucas probable-prime test with Selfridge's parameters (definition above)."""
    if n < 2:
        return False
    if n == 2:
        return True
    if n % 2 == 0 or math.isqrt(n) ** 2 == n:
        return False
    pq = selfridge(n)
    if pq is None:
        return False
    D, P, Q = pq
    d, s = n + 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    U, V, Qk = lucas_uv(P, Q, d, n)
    if U == 0 or V == 0:
        return True
    for _ in range(s - 1):
        V, Qk = (V * V - 2 * Qk) % n, Qk * Qk % n
        if V == 0:
            return True
    return False


def bpsw(n: int) -> bool:
    """The BPSW probable-prime test: the strong test to base 2 and the strong Lucas test."""
    return sprp2(n) and strong_lucas(n)


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
        if bpsw(N + X):
            return X, i + 1
    return 0, len(xs)


def surround(P: int, d: int, m: int, sl: int, bits_row=None, trial: int = 0) -> tuple[int, int, int, int]:
    """(prev, next, tests_prev, tests_next) for N = m * P#/d.

    prev = the largest X < 0 with N + X a BPSW probable prime, next = the smallest X > 0 with N + X
    a BPSW probable prime, searched only within [-sl, sl]; 0 means none there.  tests_* counts the
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
    """True iff every N + X for X in xs fails the strong test to base 2, and so BPSW (checked in
    parallel processes)."""
    N = m * plain.K_of(P, d)
    ns = [N + int(X) for X in xs]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return not any(ex.map(sprp2, ns, chunksize=max(1, len(ns) // (8 * workers))))


def limbs(n: int, n_limbs: int) -> np.ndarray:
    """n as little-endian 32-bit limbs."""
    return np.array([(n >> (32 * i)) & 0xffffffff for i in range(n_limbs)], dtype=np.uint32)

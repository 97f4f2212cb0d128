"""Pins of the probable-prime oracle (oracle/prp.py) against facts that do not come from it:
primality by trial division, theorems about base-2 strong pseudoprimes, known primes, and the two
record gaps the paper reports (Section 1)."""
import json
import os

import numpy as np
import pytest

from oracle import coracle, plain, prp

HERE = os.path.dirname(os.path.abspath(__file__))


def _trial_prime(n):
    if n < 2:
        return False
    q = 2
    while q * q <= n:
        if n % q == 0:
            return False
        q += 1
    return True


def test_agrees_with_trial_division_below_2047():
    """2047 = 23 * 89 is the smallest odd composite passing the strong test to base 2, so below it
    the test decides primality exactly."""
    for n in range(0, 2047):
        assert prp.sprp2(n) == _trial_prime(n), n


def test_strong_pseudoprimes_below_1e5():
    """There are exactly 16 strong pseudoprimes to base 2 below 10^5; the first five, factored."""
    found = [n for n in range(3, 10**5, 2) if prp.sprp2(n) and not _trial_prime(n)]
    assert len(found) == 16
    assert found[:5] == [2047, 3277, 4033, 4681, 8321]
    assert [23 * 89, 29 * 113, 37 * 109, 31 * 151, 53 * 157] == found[:5]


def test_carmichael_numbers_pass_fermat_but_fail_the_strong_test():
    for n in (561, 1105, 1729, 2465, 2821, 6601, 8911):
        assert pow(2, n - 1, n) == 1 and not _trial_prime(n)
        assert not prp.sprp2(n)


def test_mersenne_numbers():
    """2^p - 1, p prime: 2 has order p, and p | (2^p - 2)/2, so every such number passes, prime
    or not (2^11 - 1 = 23 * 89, 2^67 - 1 = 193707721 * 761838257287 are composite)."""
    for p in (61, 89, 107, 127, 521, 607, 1279):          # Mersenne primes
        assert prp.sprp2(2**p - 1)
    assert 193707721 * 761838257287 == 2**67 - 1 and prp.sprp2(2**67 - 1)
    assert 23 * 89 == 2**11 - 1 and prp.sprp2(2**11 - 1)
    # composite 2^k - 1 with k composite fail
    for k in (15, 21, 33, 35, 49, 63, 77):
        assert not prp.sprp2(2**k - 1)


def test_products_of_two_large_primes_fail():
    p, q = 2**127 - 1, 2**89 - 1
    assert not prp.sprp2(p * q)
    assert not prp.sprp2((2**61 - 1) * (2**89 - 1))


def test_candidate_order_and_columns():
    below, above = prp.candidates(211, 210, 40)
    assert below[0] == -1 and above[0] == 1
    assert all(a > b for a, b in zip(below, below[1:])) and all(a < b for a, b in zip(above, above[1:]))
    K = plain.K_of(211, 210)
    import math
    assert all(math.gcd(X, K) == 1 for X in below + above)
    # a sieved row removes marked columns
    bits = np.zeros(len(plain.columns(211, 210, 40)), dtype=np.uint8)
    bits[:] = 1
    b2, a2 = prp.candidates(211, 210, 40, bits)
    assert b2 == [] and a2 == []


def _record(i):
    """Record gap i of the paper as P, d, m, prev, next, gap, merit."""
    g = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))["record_gaps"]["gaps"][i]
    return dict(P=g["P"], d=g["d"], m=g["m"], prev=g["x_prev"], next=g["x_prev"] + g["gap"], gap=g["gap"],
                merit=g["merit"])


def test_record_gap_953():
    """The gap of 35,308 after 100054841 * 953#/210 - 9670, merit 38.048 (Section 1): with the
    row sieved to 1e8 by the oracle, the first probable primes walking out from N are at -9670 and
    +25638, and every unmarked number strictly between them fails the test."""
    r = _record(0)
    P, d, m = r["P"], r["d"], r["m"]
    sl = 26000
    bits, _ = coracle.sieve_rows(P, d, sl, [m], 2, 10**8)
    row = plain.unpack(bits, len(plain.columns(P, d, sl)))[0]
    below, above = prp.candidates(P, d, sl, row)
    ia = above.index(r["next"])
    ib = below.index(r["prev"])
    N = m * plain.K_of(P, d)
    assert prp.sprp2(N + r["prev"]) and prp.sprp2(N + r["next"])
    assert prp.interior_composite(P, d, m, below[:ib] + above[:ia])
    assert r["next"] - r["prev"] == r["gap"]
    assert round(prp.merit(P, d, m, r["prev"], r["next"]), 3) == r["merit"]


def test_record_gap_1019_endpoints():
    """The gap of 36,702 after 164065661 * 1019#/210 - 18566, merit 37.051 (Section 1): both
    endpoints pass, and the merit follows from them."""
    r = _record(1)
    N = r["m"] * plain.K_of(r["P"], r["d"])
    assert prp.sprp2(N + r["prev"]) and prp.sprp2(N + r["next"])
    assert r["next"] - r["prev"] == r["gap"]
    assert round(prp.merit(r["P"], r["d"], r["m"], r["prev"], r["next"]), 3) == r["merit"]

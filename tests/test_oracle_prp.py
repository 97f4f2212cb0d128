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


# ------------------------------------------------------------------------------------------
# Strong Lucas test and BPSW (the second half of the test the paper's search runs, Section 2.2)
# ------------------------------------------------------------------------------------------
def _primes_below(n):
    return [q for q in range(2, n) if _trial_prime(q)]


def test_jacobi_is_euler_criterion_for_primes():
    """For a prime p, (a/p) = a^((p - 1)/2) mod p (Euler's criterion), with 0 for p | a."""
    for p in _primes_below(700)[1:]:
        for a in range(-3 * p, 3 * p):
            e = pow(a % p, (p - 1) // 2, p)
            want = 0 if a % p == 0 else (1 if e == 1 else -1)
            assert prp.jacobi(a, p) == want, (a, p)


def test_jacobi_is_multiplicative_in_the_modulus():
    """(a/mn) = (a/m)(a/n) for odd m, n (the Jacobi symbol's definition as a product)."""
    for m in range(1, 90, 2):
        for n in range(1, 90, 2):
            for a in range(-40, 41):
                assert prp.jacobi(a, m * n) == prp.jacobi(a, m) * prp.jacobi(a, n)


def test_lucas_doubling_equals_the_recurrence():
    """U_k, V_k mod n from the doubling ladder equal the sequences' definition
    W_(k+1) = P W_k - Q W_(k-1), stepped one index at a time."""
    for n in (101, 1009, 65537, 2**61 - 1, 10**12 + 39):
        for P, Q in ((1, -1), (1, 2), (1, -3), (3, 5), (1, 12)):
            U0, U1, V0, V1 = 0, 1, 2, P
            for k in range(1, 300):
                U, V, Qk = prp.lucas_uv(P, Q, k, n)
                assert (U, V, Qk) == (U1 % n, V1 % n, pow(Q, k, n)), (n, P, Q, k)
                U0, U1 = U1, P * U1 - Q * U0
                V0, V1 = V1, P * V1 - Q * V0


def test_selfridge_parameters():
    """D is the first of 5, -7, 9, -11, ... with (D/n) = -1; Q = (1 - D)/4."""
    assert prp.selfridge(13) == (5, 1, -1)             # (5/13) = (13/5) = (3/5) = -1
    assert prp.selfridge(101) == (-7, 1, 2)            # (5/101) = (1/5) = 1; (-7/101) = (101/7) = (3/7) = -1
    for n in (101, 103, 107, 109, 1009, 65537, 999983):
        D, P, Q = prp.selfridge(n)
        assert prp.jacobi(D, n) == -1 and P == 1 and 4 * Q == 1 - D
        k = 5
        while abs(k) < abs(D):
            assert prp.jacobi(k, n) != -1
            k = -(k + 2) if k > 0 else -k + 2
    assert prp.selfridge(35) is None                   # (5/35) = 0 with 5 != 35: 35 is composite


def test_every_odd_prime_passes_strong_lucas():
    for p in _primes_below(10**5)[1:]:
        assert prp.strong_lucas(p), p


def test_strong_lucas_pseudoprimes_below_1e5():
    """The composites below 10^5 that pass the strong Lucas test with Selfridge's parameters
    (Baillie and Wagstaff 1980; OEIS A217255): 12 of them, none a strong pseudoprime to base 2."""
    found = [n for n in range(3, 10**5, 2) if prp.strong_lucas(n) and not _trial_prime(n)]
    assert found == [5459, 5777, 10877, 16109, 18971, 22499, 24569, 25199, 40309, 58519, 75077, 97439]
    assert [53 * 103, 53 * 109, 73 * 149] == found[:3]
    assert not any(prp.sprp2(n) for n in found)


def test_bpsw_is_primality_below_1e5():
    """BPSW has no pseudoprime below 2^64 (exhaustively verified), so below 10^5 it is exact."""
    for n in range(0, 10**5):
        assert prp.bpsw(n) == _trial_prime(n), n


def test_bpsw_rejects_base2_pseudoprimes_and_keeps_mersenne_primes():
    for n in (2047, 3277, 4033, 4681, 8321, 2**11 - 1, 2**67 - 1):
        assert prp.sprp2(n) and not prp.bpsw(n)
    for p in (61, 89, 107, 127, 521, 607, 1279):
        assert prp.bpsw(2**p - 1)
    assert not prp.bpsw((2**61 - 1) * (2**89 - 1))
    assert not prp.bpsw(1009**2) and not prp.strong_lucas((2**61 - 1)**2)   # squares


def test_surround_skips_a_base2_pseudoprime():
    """N = 68 * 5#/1 = 2040: 2047 = 23 * 89 (X = 7) passes the base-2 test; BPSW goes on to the
    prime 2053 (X = 13).  Below N, 2039 (X = -1) is prime."""
    prev, nxt, tp, tn = prp.surround(5, 1, 68, 20)
    assert (prev, nxt, tp, tn) == (-1, 13, 1, 4)      # above: 2041 = 13 * 157, 2047, 2051 = 7 * 293, 2053
    assert prp.sprp2(2040 + 7) and not prp.bpsw(2040 + 7)

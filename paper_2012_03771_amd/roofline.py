"""Algorithmic work of the large-prime branch, for its ALU roofline.

Units and their prices in VALU lane-operations (fp64 and 32/64-bit integer ops alike, one
lane-operation each; gfx950 issues fp64 FMA at the full vector rate):

  level  one level of the recursion of Eq. 5 (Section 3.3): a reciprocal of the current modulus
         good to 2^-47 (hardware seed and one Newton step: 3 ops), the remainders L mod K and
         p mod K (multiply, floor, fma: 3 ops each, exact without correction below 2^42), the
         offset K - (L mod K) with its zero case (2), the terminal test (c) (1), and the mirror
         (d): its test, the new L and K and two selects (7): 19 ops.
  solve  turning a solution value into its multiplier, t = v * k^-1 mod p: the value (1) and one
         fp64 modular multiplication (two-product, quotient, remainder, reduction: 11): 12 ops.
  hit    one m with p | m*K + X: the residue step and the gcd(m, d) / column filters (10 ops
         with a solve per hit; 14 ops with three-gap stepping, which also picks the step).
  prime  per-prime setup: k^-1 mod p and the three-gap constants by one extended Euclidean pass
         (about 20 steps of 8 ops: reciprocal 3, quotient 2, remainder 1, Bezout coefficient 1,
         test 1), the two return times (2 x 10) and the start residue (15): 195 ops; and, when
         the large branch forms K mod p itself (a single job), the product of K's prime groups
         (6 ops per group) and m_start K mod p (20 ops).

These are the minimum operation counts of the arithmetic the algorithm requires; executed
instructions are higher (exec-mask handling, address arithmetic, divergence), so the achieved
fraction they give is a lower bound of the VALU utilisation.
"""
OPS_LEVEL = 19
OPS_SOLVE = 12
OPS_HIT_G = 10
OPS_HIT_THREE_GAP = 14
OPS_PRIME = 195
OPS_KMOD_GROUP = 6
OPS_KMOD_FIXED = 20
GROUP_MAX = 1 << 50


def kmod_groups(P: int, d: int) -> int:
    """Number of products of the primes dividing K = P#/d, taken in ascending order while the
    product stays below 2^50 (the groups the K mod p chain multiplies)."""
    ps = [q for q in range(2, P + 1) if all(q % r for r in range(2, int(q ** 0.5) + 1))]
    g, n = 1, 0
    for q in ps:
        if d % q == 0:
            continue
        if g > (GROUP_MAX - 1) // q:
            n += 1
            g = q
        else:
            g *= q
    return n + (1 if g > 1 else 0)


def large_branch_ops(diag, three_gap: bool, kmod_groups_formed: int = 0) -> float:
    """kmod_groups_formed: K's group count when the large branch forms K mod p of its primes
    itself (0 when it reads the tables)."""
    hit = OPS_HIT_THREE_GAP if three_gap else OPS_HIT_G
    per_prime = OPS_PRIME + (OPS_KMOD_GROUP * kmod_groups_formed + OPS_KMOD_FIXED if kmod_groups_formed else 0)
    return (float(diag.g_levels) * OPS_LEVEL + float(diag.g_calls) * OPS_SOLVE
            + float(diag.large_raw_hits) * hit + float(diag.large_primes) * per_prime)

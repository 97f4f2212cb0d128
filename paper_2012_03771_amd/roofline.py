"""Algorithmic work of the large-prime branch, for its ALU roofline.

Units and their prices in VALU lane-operations (fp64 and 32/64-bit integer ops alike, one
lane-operation each; gfx950 issues fp64 FMA at the full vector rate):

  level  one level of the recursion of Eq. 5 (Section 3.3): a reciprocal of the current
         modulus (v_rcp + two Newton steps = 5 ops), two exact remainders L mod K and p mod K
         (multiply, floor, fma, two one-sided corrections = 8 ops each) and about 6 ops of case
         tests and state update: 27 ops.
  solve  turning a solution value into its multiplier, t = v * k^-1 mod p: one modular
         multiplication (fp64 quotient estimate, two 64-bit products, correction): 12 ops.
  hit    one m with p | m*K + X: the residue step and the gcd(m, d) / column filters (10 ops
         with a solve per hit; 14 ops with three-gap stepping, which also picks the step).
  prime  per-prime setup: k^-1 mod p by the extended Euclidean algorithm (about 20 steps of
         14 ops) plus the start residue: 310 ops.

These are the minimum operation counts of the arithmetic the algorithm requires; executed
instructions are higher (exec-mask handling, address arithmetic, divergence), so the achieved
fraction they give is a lower bound of the VALU utilisation.
"""
OPS_LEVEL = 27
OPS_SOLVE = 12
OPS_HIT_G = 10
OPS_HIT_THREE_GAP = 14
OPS_PRIME = 310


def large_branch_ops(diag, three_gap: bool) -> float:
    hit = OPS_HIT_THREE_GAP if three_gap else OPS_HIT_G
    return (float(diag.g_levels) * OPS_LEVEL + float(diag.g_calls) * OPS_SOLVE
            + float(diag.large_raw_hits) * hit + float(diag.large_primes) * OPS_PRIME)

"""Algorithmic work of the large-prime branch, for its ALU roofline.

The unit of work is one level of the recursion of Eq. 5 (Section 3.3).  Each level costs a
fixed number of VALU lane-operations in this implementation's level body: an fp64 reciprocal
of the current modulus and up to two exact remainders (L mod K, p mod K), the case tests and
the state update.  OPS_PER_LEVEL is that straight-line count, read from the gfx950 assembly of
the kernel (the (e) case, the most frequent one).  Work outside the levels (per-solve inverse
multiplication, per-prime inverse, hit recording) is not counted, so the figure is a lower
bound of the work actually done.
"""
OPS_PER_LEVEL = 52


def large_branch_ops(diag) -> float:
    return float(diag.g_levels) * OPS_PER_LEVEL

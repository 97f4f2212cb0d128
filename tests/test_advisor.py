"""CPU pins of the parameter advisor's formulas (Section 4): Eq. 6 against the theoretical column
of Section 4.1's table, Eq. 7 against the expected primality tests of Table A.1 (Appendix), and
log(P#) against Table A.1's second column."""
import json
import math
import os

import pytest

from paper_2012_03771_amd import advisor as A

HERE = os.path.dirname(os.path.abspath(__file__))

# Table A.1 (Appendix, experimental sieve limits): P, log(P#), sieve limit, expected tests
TABLE_A1 = [(1511, 1469, 250e9, 31.5), (4441, 4353, 2000e9, 86.3), (5333, 5228, 2000e9, 103.7),
            (8887, 8779, 1000e9, 178.4)]


def test_eq6_matches_section_4_1_theoretical_column(paper_values):
    for lim, printed in paper_values["mertens_theoretical"].items():
        if lim.startswith("_"):
            continue
        digits = len(printed.split(".")[1])
        assert round(A.mertens_fraction(float(lim)), digits) == pytest.approx(float(printed), abs=10 ** -digits), lim


@pytest.mark.parametrize("P,log_primorial,limit,expected", TABLE_A1)
def test_eq7_matches_table_a1(P, log_primorial, limit, expected):
    theta = sum(math.log(q) for q in A._primes_upto(P))
    assert round(theta) == log_primorial
    assert A.expected_tests(log_primorial, limit) == pytest.approx(expected, abs=0.1)


def test_table_a1_row_2221_is_inconsistent():
    """The 2221 row prints log(P#) = 2054 and 40.9 tests at 800e9; log(2221#) is 2154 and Eq. 7 gives
    44.1 with it (42.1 with 2054): the row is taken as misprinted."""
    theta = sum(math.log(q) for q in A._primes_upto(2221))
    assert round(theta) == 2154
    assert abs(A.expected_tests(theta, 800e9) - 40.9) > 1 and abs(A.expected_tests(2054, 800e9) - 40.9) > 1


def test_expected_tests_shrink_with_the_limit():
    e = [A.expected_tests(929.0, 10.0 ** k) for k in range(4, 14)]
    assert all(a > b for a, b in zip(e, e[1:]))
    # sieving 10x deeper saves the fraction 1 - log(L)/log(10 L) of the tests
    assert e[0] / e[1] == pytest.approx(5.0 / 4.0)


def test_interval_range_and_log_n():
    import workloads as W
    ln = A.log_n_of(W.PAPER_SCALE)
    from oracle import plain
    assert ln == pytest.approx(math.log(plain.K_of(953, 210) * 10**8), rel=1e-12)
    lo, hi = A.interval_range(ln)
    assert lo == math.ceil(6 * ln) and hi == math.floor(10 * ln)
    assert lo <= W.PAPER_SCALE.sl <= hi * 4

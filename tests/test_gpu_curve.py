"""The combined-sieve speedup curve of bench.py (Section 3's speedup figure): the one-interval
sieve with every prime in the per-interval branch and the combined sieve agree bit for bit on
sampled rows, and the speedup grows with the number of intervals."""
import argparse
import os
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_mc_curve_small_limit():
    import numpy as np
    import bench
    import workloads as W
    import paper_2012_03771_amd as cs
    print("mc curve, limit 1e8", flush=True)
    args = argparse.Namespace(curve_limit=10**8, curve_mc="1,100,2000")
    out = bench._mc_curve(cs, torch, W, np, args)
    pts = out["points"]
    assert [p["m_c"] for p in pts] == [1, 100, 2000]
    assert out["rows_checked"]["identical"] and out["rows_checked"]["m_c"] == 2000
    sp = [p["speedup"] for p in pts]
    assert sp[0] < sp[1] < sp[2]
    # every interval has about the same number of factors: the total grows with M_c
    f = [p["factors"] / p["m_c"] for p in pts]
    assert max(f) < 1.1 * min(f)

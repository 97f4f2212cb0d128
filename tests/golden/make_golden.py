"""Writes the stored oracle results used by the GPU parity tests at full job sizes.

Every value written here comes from oracle/ (the plain CPU sieve) on jobs from workloads/;
nothing comes from the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py [medium] [paper] [batch] [wide]

medium_503_rows.npz   per-row digests of the whole 503#/210 job (2,287 rows), plus 64 full rows
paper_953_rows.npz    64 rows of the 953#/210 paper-scale job, primes up to 1e10: the first, the
                      last, the row of m = 100054841 (the merit-38.048 record gap) and 61 seeded
batch_rows.npz        4 rows of each of the 64 seeded mixed-batch jobs
wide_windows.npz      every row of two jobs placed on windows of primes near 2^50 and 2^63

Every file is written with the oracle's DIRECT mode: N mod p taken from the bignum N = m K for
every row and prime, the traditional sieve of Section 2.1 written out, so that no stored value
relies on the (m mod p)(K mod p) identity of Eq. 1 that the GPU path itself uses.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import workloads as W  # noqa: E402
from oracle import coracle  # noqa: E402
from goldens import row_digests  # noqa: E402


def medium():
    job = W.MEDIUM
    t = time.time()
    ms = coracle.rows(job.d, job.m_start, job.m_inc)
    bits, counts = coracle.sieve_rows(job.P, job.d, job.sl, ms, 2, job.limit, mode=coracle.DIRECT)
    full = W.sample_rows(len(ms), 64, seed=21)
    np.savez_compressed(os.path.join(HERE, "medium_503_rows.npz"), job=np.array(job.as_tuple(), dtype=np.uint64),
                        digests=row_digests(bits, counts), rows=np.array(full), bits=bits[full],
                        counts=counts[full], total_factors=np.uint64(counts.sum()))
    print(f"medium: {len(ms)} rows in {time.time() - t:.1f} s, {int(counts.sum())} factors")


def paper():
    job = W.PAPER_SCALE
    t = time.time()
    ms = coracle.rows(job.d, job.m_start, job.m_inc)
    rec = W.RECORD_GAPS[0][2]
    r_rec = int(np.searchsorted(ms, rec))
    assert ms[r_rec] == rec
    rows = W.sample_rows(len(ms), 64, seed=31, must=[r_rec])
    bits, counts = coracle.sieve_rows(job.P, job.d, job.sl, ms[rows], 2, job.limit, mode=coracle.DIRECT)
    np.savez_compressed(os.path.join(HERE, "paper_953_rows.npz"), job=np.array(job.as_tuple(), dtype=np.uint64),
                        rows=np.array(rows), m=ms[rows], bits=bits, counts=counts, record_row=np.int64(r_rec))
    print(f"paper: {len(rows)} rows in {time.time() - t:.1f} s")


def batch():
    jobs = W.batch_jobs(64, seed=0)
    t = time.time()
    out = {}
    for i, job in enumerate(jobs):
        ms = coracle.rows(job.d, job.m_start, job.m_inc)
        if len(ms) == 0:
            continue
        rows = W.sample_rows(len(ms), 4, seed=100 + i)
        bits, counts = coracle.sieve_rows(job.P, job.d, job.sl, ms[rows], 2, job.limit, mode=coracle.DIRECT)
        out[f"job{i}_rows"] = np.array(rows)
        out[f"job{i}_bits"] = bits
        out[f"job{i}_counts"] = counts
        out[f"job{i}_tuple"] = np.array(job.as_tuple(), dtype=np.uint64)
        print(f"  batch job {i}: {job} rows={len(ms)} ({time.time() - t:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "batch_rows.npz"), **out)
    print(f"batch: 64 jobs in {time.time() - t:.1f} s")


def wide():
    """Windows of the prime range near 2^50 and just below 2^63, where the GPU takes its exact
    64-bit residue path.  Large primes hit an interval of a feasible job there with probability
    about rows * S / p, so each job is placed where a chosen prime q of its window does divide:
    K = 7# (P = 7, d = 1), q the first prime at or above the window's centre (from the oracle's
    sieve), and m0 = -K^-1 mod q, so that q divides m K + X for X = 1 + 210 j at m = m0 - j: 39
    rows of the 1,000 hold a factor q at a column (|X| <= 4000, X = 1 mod 210 is coprime to K).
    Expected bitmaps and counts: the oracle's direct sieve of every row with every prime of the
    window.  Only the job's placement uses Python integers; no expected value does."""
    out = {}
    for name, centre in (("w50", 1 << 50), ("w63", (1 << 63) - (1 << 23))):
        t = time.time()
        q = int(coracle.primes_range(centre, centre + 10**5)[0])
        K = 210
        m0 = (-pow(K, -1, q)) % q
        job = W.Job(7, 1, m0 - 500, 1000, 4000, q + (1 << 22))
        p_lo, p_hi = q - (1 << 22), q + (1 << 22)
        ms = coracle.rows(job.d, job.m_start, job.m_inc)
        bits, counts = coracle.sieve_rows(job.P, job.d, job.sl, ms, p_lo, p_hi, mode=coracle.DIRECT)
        n_pr = len(coracle.primes_range(p_lo, p_hi))
        out[f"{name}_job"] = np.array(job.as_tuple(), dtype=np.uint64)
        out[f"{name}_window"] = np.array([p_lo, p_hi, q, n_pr], dtype=np.uint64)
        out[f"{name}_bits"] = bits
        out[f"{name}_counts"] = counts
        print(f"wide {name}: q={q} m0={m0} primes in window {n_pr} factors {int(counts.sum())} "
              f"({time.time() - t:.1f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "wide_windows.npz"), **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["medium", "paper", "batch", "wide"]
    for w in which:
        {"medium": medium, "paper": paper, "batch": batch, "wide": wide}[w]()

"""Benchmark of the Combined Sieve hot path on one MI355X.

A step is one whole cs_sieve call on the paper-scale job 953#/210, m in [1e8, 1e8 + 1e6),
sl = 20000, primes up to 1e10: prime table, K mod p for all 455,052,511 primes, row/column
maps, the small-prime branch and the large-prime branch, with every input built on the device
inside the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "factors found/s + primes/s on 953#/210 sieve; served-job p50/p99 latency"

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz -> 39.3e12 VALU lane-operations per second
# (the fp64 FMA rate, 78.6 TFLOP/s, counts two flops per such operation).
ALU_PEAK_OPS = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12
# v_mad_u64_u32 (32 x 32 -> 64-bit multiply-add, the limb product of the probable-prime test)
# issues at the full VALU rate on gfx950 (an independent-chain probe measured 3.4e13/s).
MAD_PEAK = 256 * 64 * 2.4e9


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", choices=["g", "three_gap"], default="three_gap")
    ap.add_argument("--scatter", choices=["auto", "atomic", "bytes", "list"], default="auto",
                    help="large-prime hit scatter of the timed step (cs_tune.scatter)")
    ap.add_argument("--thr-mult", type=float, default=0.0,
                    help="small/large threshold of the timed step as a multiple of S = 2 sl + 1 (0: the plan's)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--cpu-rows", type=int, default=8,
                    help="rows of the job the oracle sieves with every prime up to the job's limit")
    ap.add_argument("--workload", default="paper_953")
    ap.add_argument("--phase-only", action="store_true", help="time the phases once, no steps")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-job batched leg")
    ap.add_argument("--no-autotune", action="store_true", help="batch leg with default tunings")
    ap.add_argument("--traffic-gb", type=float, default=None,
                    help="HBM traffic of one k_large launch from the committed FETCH_SIZE/WRITE_SIZE profile "
                         "of the same kernel (GB), reported as roofline.traffic")
    ap.add_argument("--no-g", action="store_true",
                    help="skip timing the phases with one Eq. 5 solve per hit (the paper's enumeration, g_mode)")
    ap.add_argument("--no-serve", action="store_true", help="skip the served (Poisson) leg")
    ap.add_argument("--serve-jobs", type=int, default=512)
    ap.add_argument("--serve-warmup", type=int, default=32)
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95",
                    help="loads (fractions of the saturated throughput) of the served legs; 0.8 is the headline")
    ap.add_argument("--serve-chunks", type=int, default=1,
                    help="large-prime chunks per served job (cs_server_config.chunks; 1 measured best on this "
                         "mix: p50 24 / p99 141 ms at 0.8 load, against 28 / 271 ms with about 2 ms of estimated "
                         "device time per chunk)")
    ap.add_argument("--serve-long-ms", type=float, default=3.0,
                    help="cs_server_config.long_ms: jobs estimated to take longer alone run in a second lane "
                         "(0: one lane; 3 measured best on this mix: p50/p99 23.6/103 ms at 0.8 load and "
                         "68/173 ms at 0.95, against 22.3/117 and 120/214 ms with one lane)")
    ap.add_argument("--prp-rows", type=int, default=16384,
                    help="rows of the sieved job searched for their surrounding probable primes (0: skip)")
    ap.add_argument("--no-atomic-probe", action="store_true",
                    help="skip the random-atomics rate probe that the roofline of the byte-counter scatter uses")
    ap.add_argument("--scatter-table", action="store_true",
                    help="instead of the step benchmark: the scatter-rate probe over buffer sizes and modes")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of this many MiB (a known-size reference for "
                         "HBM byte counters)")
    ap.add_argument("--mc-curve", action="store_true",
                    help="instead of the step benchmark: speedup of the combined sieve over a per-interval "
                         "sieve against the number of intervals M_c (K = 1511#/7#, X = 18,000)")
    ap.add_argument("--table-a2", action="store_true",
                    help="instead of the step benchmark: configurations of the paper's amortized runtime "
                         "table (row 10: 1511#/(7#*1009), X = 16,000, M = 1e7, primes to 1e11)")
    ap.add_argument("--a2-rows", default="10", help="rows of that table: any of 10, 11, 12, 15")
    ap.add_argument("--curve-limit", type=int, default=10**11)
    ap.add_argument("--curve-mc", default="1,10,100,1000,10000,100000,1000000")
    return ap.parse_args()


# The paper's amortized-runtime table (Appendix, Table A.2): (P, d, X, M, limit, seconds per coprime m).
TABLE_A2 = {
    10: (1511, 2 * 3 * 5 * 7 * 1009, 16000, 10**7, 10**11, 0.0112),
    11: (1511, 2 * 3 * 5 * 7 * 1009, 16000, 10**7, 25 * 10**10, 0.0129),
    12: (2221, 2 * 3 * 5 * 2027, 23000, 10**7, 8 * 10**11, 0.0252),
    13: (4441, 2 * 3 * 5 * 7 * 11 * 4001, 47000, 10**7, 2 * 10**12, 0.0605),
    14: (5333, 2 * 3 * 5 * 7 * 11 * 5003, 65000, 10**6, 2 * 10**12, 0.158),
    15: (8887, 2 * 3 * 5 * 7 * 11 * 13 * 17 * 8009, 100000, 10**5, 10**12, 0.709),
}


def _table_a2(cs, torch, W, rows):
    """Rows of the paper's amortized-runtime table (Appendix, Table A.2): K = P#/d with d of a
    large prime factor (rows come from the dense m -> row table), M multipliers from m = 1, every
    prime up to the limit.  Where the whole prime, K mod p and m_start*K mod p tables would exceed
    160 GiB the prime range is taken in chunks of 2^36 integers (cs_sieve_chunked).  One call
    timed after a warm-up call.  The paper's seconds per coprime m come from a CPU whose type it
    does not state."""
    out = []
    for r in rows:
        P, d, X, M, limit, paper = TABLE_A2[r]
        job = W.Job(P, d, 1, M, X, limit)
        tune = cs.Tune(large_mode=cs.LARGE_THREE_GAP)
        s = torch.cuda.current_stream()
        whole = cs.plan(job, tune)
        span = 1 << 36 if whole.ws_bytes > (160 << 30) else 0
        lay = cs.plan_chunked(job, span, tune) if span else whole
        print(f"# table A.2 row {r}: rows {lay.n_m} cols {lay.n_x} ws {lay.ws_bytes / 2**30:.1f} GiB"
              f" chunks of {span or limit + 1:.3g}", file=sys.stderr, flush=True)
        bitmap = torch.empty((lay.n_m, lay.row_words), dtype=torch.int32, device="cuda")
        counts = torch.empty((lay.n_m,), dtype=torch.int32, device="cuda")
        ws = torch.empty((lay.ws_bytes,), dtype=torch.uint8, device="cuda")

        def run():
            if span:
                cs.sieve_chunked_into(job, span, bitmap, counts, ws, tune, s)
            else:
                cs.sieve_into(job, bitmap, counts, ws, tune, s)
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        factors = int(counts.to(torch.int64).sum().item())
        dg = cs.diag_read(ws, s)
        out.append({"row": r, "s_per_m": t / lay.n_m, "total_s": t, "paper_s_per_m": paper,
                    "config": {"P": P, "d": d, "sl": X, "m_start": 1, "m_inc": M, "limit": limit, "rows": lay.n_m,
                               "cols": lay.n_x, "thr": lay.thr, "scatter": lay.scatter, "span": span},
                    "factors": factors, "factors_per_s": factors / t, "n_primes": dg.n_primes,
                    "primes_per_s": dg.n_primes / t})
        print(f"# row {r}: {t:.3f} s, {t / lay.n_m * 1e6:.3f} us per m (paper {paper} s)", file=sys.stderr, flush=True)
        del bitmap, counts, ws
        torch.cuda.empty_cache()
    return {"metric": "sieve time per coprime m", "unit": "s", "n_gpus": 1,
            "workload": "rows of the paper's amortized-runtime table, m from 1",
            "paper_hardware": "not stated (CPU)", "rows": out}


def _mc_curve(cs, torch, W, np, args):
    """Speedup of the Combined Sieve over sieving each interval on its own, against M_c, on the
    configuration of the paper's speedup figure (Section 3: K = 1511#/7#, X = 18,000,
    P_limit = 1e11).  The per-interval sieve is this library on a job of one interval with every
    prime below the threshold: K mod p is taken for every prime and every multiple is marked from
    the residue, which is the traditional sieve's work for one interval.  The prime table is a
    one-time cost shared by any number of intervals in both methods and is left out of both
    times.  speedup(M_c) = M_c * T(one interval) / T(M_c intervals)."""
    P, d, sl, limit = 1511, 210, 18000, args.curve_limit
    mcs = [int(x) for x in args.curve_mc.split(",")]
    s = torch.cuda.current_stream()

    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    tp = timed(lambda: cs.primes(limit, s))
    torch.cuda.empty_cache()
    print(f"# curve: prime table to {limit:.3g} {tp * 1e3:.1f} ms", file=sys.stderr, flush=True)

    def m_inc_for(mc):      # smallest M with mc multipliers in [1, M] coprime to d
        phi = sum(1 for r in range(d) if math.gcd(r, d) == 1)
        M = (mc // phi) * d
        c = (mc // phi) * phi
        while c < mc:
            M += 1
            if math.gcd(M, d) == 1:
                c += 1
        return max(M, 1)

    def run(job, tune):
        lay, bitmap, counts, ws = cs.binding.alloc_outputs(job, tune)
        t = timed(lambda: cs.sieve_into(job, bitmap, counts, ws, tune, s))
        return t, lay, bitmap, counts, ws

    # one interval, every prime in the per-interval (small) branch
    one = W.Job(P, d, 1, 1, sl, limit)
    t1, lay1, *_ = run(one, cs.Tune(thr=limit))
    torch.cuda.empty_cache()
    per_interval = t1 - tp
    print(f"# curve: one interval {t1 * 1e3:.1f} ms ({per_interval * 1e3:.1f} ms without the prime table)",
          file=sys.stderr, flush=True)
    points = []
    check = None
    for mc in mcs:
        job = W.Job(P, d, 1, m_inc_for(mc), sl, limit)
        t, lay, bitmap, counts, ws = run(job, cs.Tune(large_mode=cs.LARGE_THREE_GAP))
        comb = t - tp
        pt = {"m_c": lay.n_m, "m_inc": job.m_inc, "ms": t * 1e3, "ms_without_primes": comb * 1e3,
              "speedup": lay.n_m * per_interval / comb, "factors": int(counts.to(torch.int64).sum().item())}
        points.append(pt)
        print(f"# curve: M_c {lay.n_m} {t * 1e3:.1f} ms speedup {pt['speedup']:.0f}", file=sys.stderr, flush=True)
        want = None
        if check is None and lay.n_m >= 1000:
            ms = cs.rows(job)
            idx = [0, lay.n_m // 2, lay.n_m - 1]
            want = ([int(ms[i]) for i in idx], bitmap[idx].cpu(), counts[idx].cpu())
        del bitmap, counts, ws
        torch.cuda.empty_cache()
        if want is not None:
            # the two enumerations agree bit for bit: sampled rows against one-interval runs of their m
            ok = True
            for k, m in enumerate(want[0]):
                o = W.Job(P, d, m, 1, sl, limit)
                b1, c1, w1 = cs.sieve(o, cs.Tune(thr=limit), s)
                ok = ok and torch.equal(b1.cpu()[0], want[1][k]) and int(c1[0].item()) == int(want[2][k].item())
                del b1, c1, w1
                torch.cuda.empty_cache()
            check = {"m_c": lay.n_m, "rows": want[0], "identical": ok}
    return {"metric": "combined-sieve speedup over a per-interval sieve", "unit": "x", "n_gpus": 1,
            "config": {"workload": "1511#/7#, X = 18000, m_start = 1", "P": P, "d": d, "sl": sl, "limit": limit},
            "prime_table_ms": tp * 1e3, "one_interval_ms": t1 * 1e3, "per_interval_ms": per_interval * 1e3,
            "points": points, "rows_checked": check}


# Host threads of the CPU baseline: the host CPU share that the measurement box allots to one GPU
# (16), or fewer where the process may use fewer cores.
CPU_SHARE = 16


def _cpu_baseline(job, n_rows, gpu_counts=None):
    """The oracle as it stands (plain per-interval sieve, bignum N mod p for every row and prime,
    Section 2.1) on a bounded sample of the workload itself: n_rows whole rows (the record-gap row
    first, then the first rows), every prime up to the job's limit.  The oracle runs over rows; to
    spread one row over the host threads its documented prime-range restriction is used: the range
    [2, limit] is cut into windows of equal width, one oracle call per window, and the windows'
    marks are OR-ed and their factors summed, which is the same definition restricted and
    recombined.  Returns the oracle's factors/s on the sample and the whole job's time at that
    rate (extrapolated, not measured)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import workloads as W
    from oracle import coracle
    import paper_2012_03771_amd as cs
    lay = cs.plan(job)
    ms_all = cs.rows(job)
    rec = W.RECORD_GAPS[0]
    pick = []
    if (job.P, job.d) == (rec[0], rec[1]) and job.m_start <= rec[2] < job.m_start + job.m_inc:
        pick.append(int(np.searchsorted(ms_all, rec[2])))
    r = 0
    while len(pick) < min(n_rows, lay.n_m):
        if r not in pick:
            pick.append(r)
        r += 1
    ms = ms_all[pick]
    threads = max(1, min(len(os.sched_getaffinity(0)), CPU_SHARE))
    n_win = 4 * threads
    edges = [2] + [2 + (job.limit - 2) * (i + 1) // n_win for i in range(n_win)]
    wins = [(edges[i] + (1 if i else 0), edges[i + 1]) for i in range(n_win)]

    def one(w):
        return coracle.sieve_rows(job.P, job.d, job.sl, ms, w[0], w[1], mode=coracle.DIRECT, threads=1)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(one, wins))
    dt = time.perf_counter() - t0
    bits = parts[0][0].copy()
    counts = parts[0][1].astype(np.uint64)
    for b, c in parts[1:]:
        bits |= b
        counts += c.astype(np.uint64)
    factors = int(counts.sum())
    out = {"value": factors / dt, "unit": "factors/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(ms)} whole rows of {lay.n_m} (m = {', '.join(str(int(m)) for m in ms)}), every prime "
                     f"<= {job.limit}, plain per-interval sieve with bignum N mod p (direct mode), the prime "
                     f"range in {n_win} windows over {threads} threads, {dt:.1f} s wall",
           "sample_factors": factors, "sample_s": dt,
           "extrapolated_job_s": dt * lay.n_m / len(ms),
           "extrapolated_note": "the whole job at the sample's per-row time (not measured)"}
    if gpu_counts is not None:
        out["rows_equal_gpu"] = bool(np.array_equal(counts.astype(np.uint32), gpu_counts[pick]))
    return out


def _scatter_probe(cs, torch, n_words, n_ops, slices=1, op=0, seed=7):
    """Rate of 32-bit operations at pseudo-random words of an n_words buffer (cs_probe_scatter: the
    words come from a hash in registers, no index loads).  op 0 = device-scope atomic add (the
    byte-counter scatter's operation), 1 = plain store, 2 = LDS atomic add; slices = 8 keeps each
    XCD on its own eighth of the buffer.  Timed with HIP events on the launch stream after one
    warm-up launch.  Returns operations per second."""
    s = torch.cuda.current_stream()
    buf = torch.zeros(n_words, dtype=torch.int32, device="cuda")
    cs.probe_scatter(buf, n_ops, slices, op, seed, s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    cs.probe_scatter(buf, n_ops, slices, op, seed + 1, s)
    e1.record(s)
    torch.cuda.synchronize()
    if op in (0, 2):
        assert int(buf.to(torch.int64).sum().item()) == 2 * n_ops, "probe lost operations"
    rate = n_ops / (e0.elapsed_time(e1) / 1e3)
    del buf
    torch.cuda.empty_cache()
    return rate


def _scatter_table(cs, torch):
    """The probe over the buffer sizes and modes that bound the hit scatters."""
    rows = []
    for mib, slices, op in [(3 * 1024, 1, 0), (3 * 1024, 8, 0), (1024, 1, 0), (256, 1, 0), (256, 8, 0), (64, 1, 0),
                            (16, 8, 0), (3 * 1024, 1, 1), (3 * 1024, 8, 1), (256, 1, 1), (16, 8, 1), (1, 1, 2)]:
        n_words = mib * 2**20 // 4
        n_ops = 1 << 28
        r = _scatter_probe(cs, torch, n_words, n_ops, slices, op)
        rows.append({"MiB": mib, "slices": slices, "op": ["atomic_add", "store", "lds_atomic_add"][op],
                     "ops_per_s": r})
        print(f"# probe {mib} MiB slices {slices} op {op}: {r:.3e}/s", file=sys.stderr, flush=True)
    return rows


def _kernel_profile(mode):
    """The committed rocprofv3 counters of one k_large launch (profiles/traffic.json), or None when
    the kernel sources changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(mode)
    m = hashlib.sha256()
    for f in ("kernels.hip", "arith.h", "arith_wide.h", "device.h"):
        m.update(open(os.path.join(ROOT, "paper_2012_03771_amd", "csrc", f), "rb").read())
    if not rec or rec.get("hash") != m.hexdigest()[:16]:
        return None
    return rec


def _kernel_traffic(mode):
    """HBM bytes (GB) of one k_large launch from the committed FETCH_SIZE/WRITE_SIZE profile."""
    rec = _kernel_profile(mode)
    return rec["traffic_gb"] if rec else None


def _valu_issue(mode):
    """Measured VALU issue of one k_large launch: SQ_INSTS_VALU (wavefront instructions, each
    occupying a 16-lane SIMD for 4 cycles) x 4 over the SIMD cycles of the launch (1,024 SIMDs at
    2.4 GHz times its duration), from the committed SQ-counter profile; None when stale."""
    rec = _kernel_profile(mode)
    return rec.get("valu_issue_frac") if rec else None


def _prp_leg(cs, torch, np, job, bitmap, n_rows, stream):
    """Surrounding probable primes of the first n_rows sieved rows (cs_surround): each side of a
    row is searched outward among its unmarked columns with the strong base-2 test, and the number
    found is checked with the strong Lucas test (BPSW)."""
    ms = cs.rows(job)[:n_rows]
    m_dev = torch.from_numpy(ms.astype(np.int64)).cuda()
    rows = bitmap[:n_rows]
    ws = torch.empty((cs.surround_ws_bytes(job, n_rows),), dtype=torch.uint8, device="cuda")
    cs.surround(job, rows, m_dev, ws, stream)                       # warm-up
    t0 = time.perf_counter()
    out, st = cs.surround(job, rows, m_dev, ws, stream)
    t1 = time.perf_counter()
    o = out.cpu().numpy().astype(np.int64)
    useful = int(o[:, 2:].sum())
    both = (o[:, 0] != 0) & (o[:, 1] != 0)
    gaps = (o[:, 1] - o[:, 0])[both]
    # algorithmic multiply-adds of one test: one Montgomery squaring (2 NL^2 limb products, CIOS)
    # per bit of N - 1 below the top one
    mads = st.tests * (st.bits - 1) * 2 * st.limbs ** 2
    sec = t1 - t0
    return {"rows": n_rows, "s": sec, "rows_per_s": n_rows / sec, "useful_tests": useful,
            "tests_run": st.tests, "tests_per_s": st.tests / sec, "useful_tests_per_s": useful / sec,
            "rounds": st.rounds, "limbs": st.limbs, "bits": st.bits, "rows_both_found": int(both.sum()),
            "mean_gap": float(gaps.mean()) if len(gaps) else None, "max_gap": int(gaps.max()) if len(gaps) else None,
            "lucas_tests": st.lucas_tests, "lucas_passes": st.lucas_passes, "lucas_ms": st.lucas_ms,
            "roofline": {"bound": "alu", "kernel": "k_sv_test", "achieved": mads / (st.test_ms / 1e3) / 1e12,
                         "peak": MAD_PEAK / 1e12, "unit": "T v_mad_u64_u32/s",
                         "frac": mads / (st.test_ms / 1e3) / MAD_PEAK, "test_ms": st.test_ms, "traffic": None}}


def _batch_leg(cs, torch, W, mode, reps=3, autotune=True):
    """64 seeded mixed jobs: one fused launch sequence replayed from a hipGraph, against 64
    sequential cs_sieve calls on the same GPU (both with the same tunings)."""
    jobs = W.batch_jobs(64, seed=0)
    t_tune = 0.0
    n_buckets = 0
    opts = {"path": cs.BATCH_AUTO}
    batch_timings = []
    if autotune:
        from paper_2012_03771_amd.autotune import Autotuner
        t0 = time.perf_counter()
        tuner = Autotuner()
        tunes, opts, batch_timings = tuner.tune_batch(jobs)
        t_tune = time.perf_counter() - t0
        n_buckets = len(tuner.cache)
    else:
        tunes = [cs.Tune(large_mode=mode) for _ in jobs]

    def timed_batch(o):
        b = cs.Batch(jobs, tunes, **o)
        bm, ct = b.alloc_outputs()
        b.run(bm, ct, use_graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.run(bm, ct, use_graph=True)
        torch.cuda.synchronize()
        return b, bm, ct, (time.perf_counter() - t0) / reps

    batch, bm, ct, t_batch = timed_batch(opts)
    path = batch.path
    factors = sum(int(c.to(torch.int64).sum().item()) for c in ct)
    diag = batch.diag()
    # the other path with the same tunings, for the comparison
    other = cs.BATCH_LANES if path == cs.BATCH_PERSISTENT else cs.BATCH_PERSISTENT
    t_other = None
    try:
        b2, bm2, ct2, t_other = timed_batch({"path": other})
        same_paths = all(torch.equal(a, b) for a, b in zip(bm, bm2)) and all(torch.equal(a, b) for a, b in zip(ct, ct2))
        b2.close()
        del bm2, ct2
    except cs.CsError:
        same_paths = None
    # the same jobs, one plain launch sequence each, one after the other
    lays = [cs.plan(j, t) for j, t in zip(jobs, tunes)]
    ws = torch.empty((max(L.ws_bytes for L in lays),), dtype=torch.uint8, device="cuda")
    sb = [torch.empty((L.n_m, L.row_words), dtype=torch.int32, device="cuda") for L in lays]
    sc = [torch.empty((L.n_m,), dtype=torch.int32, device="cuda") for L in lays]
    for i, j in enumerate(jobs):
        cs.sieve_into(j, sb[i], sc[i], ws, tunes[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for i, j in enumerate(jobs):
            cs.sieve_into(j, sb[i], sc[i], ws, tunes[i])
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / reps
    same = all(torch.equal(a, b) for a, b in zip(bm, sb)) and all(torch.equal(a, b) for a, b in zip(ct, sc))
    batch.close()
    del bm, ct, sb, sc, ws
    torch.cuda.empty_cache()
    return {"workload": "64 seeded mixed jobs (P in primes [307,1019], d in {1,2,6,30,210}, m_inc 1e3-1e5, "
                        "limit 1e7-1e9, sl = round(40 ln N))",
            "path": {cs.BATCH_PERSISTENT: "persistent", cs.BATCH_LANES: "lanes"}[path],
            "items_per_task": opts.get("items_per_task") or None,
            "ms_other_path": t_other * 1e3 if t_other is not None else None, "other_path_identical": same_paths,
            "autotune_batch_ms": batch_timings,
            "ms_batched": t_batch * 1e3, "ms_sequential": t_seq * 1e3, "speedup": t_seq / t_batch,
            "jobs_per_s": 64 / t_batch, "factors_per_s": factors / t_batch,
            "seq_jobs_per_s": 64 / t_seq, "factors": factors, "identical_to_sequential": bool(same),
            "primes_in_shared_table": diag.n_primes, "autotuned": autotune, "autotune_buckets": n_buckets,
            "autotune_s": t_tune}


def _server_capacity(cs, W, mode, n_jobs=128, chunks=1, long_ms=0.0):
    """Saturated throughput of the server: n_jobs from the mixed-batch distribution (seed 2)
    submitted at once, completed jobs per second."""
    _, jobs = W.poisson_arrivals(n_jobs, 1.0, seed=2)
    srv = cs.Server(budget_bytes=64 << 30, max_limit=max(j.limit for j in jobs), max_active=32, chunks=chunks,
                    tune=cs.Tune(large_mode=mode), long_ms=long_ms)
    t0 = time.perf_counter()
    tickets = [srv.submit(j) for j in jobs]
    for t in tickets:
        srv.wait(t, 600.0)
        srv.release(t)
    span = time.perf_counter() - t0
    srv.close()
    return n_jobs / span


def _alone_times(cs, torch, W, mode, n_jobs):
    """Device time of each of the first n_jobs jobs of the served stream run alone (cs_sieve on the
    current stream, HIP events around it): the service times queueing adds to."""
    import numpy as np
    _, jobs = W.poisson_arrivals(n_jobs, 1.0, seed=1)
    s = torch.cuda.current_stream()
    out = []
    for job in jobs:
        tune = cs.Tune(large_mode=mode)
        lay, bm, ct, ws = cs.binding.alloc_outputs(job, tune)
        cs.sieve_into(job, bm, ct, ws, tune, s)                       # warm-up (first use of the sizes)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        cs.sieve_into(job, bm, ct, ws, tune, s)
        e1.record(s)
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
        del bm, ct, ws
    torch.cuda.empty_cache()
    a = np.array(out)
    return {"jobs": n_jobs, "p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean()), "max_ms": float(a.max())}


def _serve_leg(cs, torch, W, mode, rate, n_jobs, n_warm, chunks=1, long_ms=0.0):
    """Poisson arrivals of jobs from the mixed-batch distribution into the continuous-batching
    server (64 GB budget); latency = completion - arrival."""
    import numpy as np
    times, jobs = W.poisson_arrivals(n_warm + n_jobs, rate, seed=1)
    srv = cs.Server(budget_bytes=64 << 30, max_limit=max(j.limit for j in jobs), max_active=32, chunks=chunks,
                    tune=cs.Tune(large_mode=mode), long_ms=long_ms)
    tickets = []
    t0 = time.perf_counter()
    for t_arr, job in zip(times, jobs):
        delay = t_arr - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(job))
    lat, factors = [], 0
    t_first = None
    for i, t in enumerate(tickets):
        info = srv.wait(t, 600.0)
        if i >= n_warm:
            lat.append(info.latency_s)
            if t_first is None:
                t_first = times[i]
            _, c = srv.fetch(t)
            factors += int(c.to(torch.int64).sum().item())
        srv.release(t)
    t_end = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    span = t_end - t_first
    lat = np.array(lat)
    return {"workload": f"{n_jobs} jobs (+{n_warm} warm-up) from the mixed-batch distribution, Poisson arrivals "
                        f"at {rate:.1f} jobs/s, 64 GB admission budget, 32 slots, "
                        f"{chunks} large-prime chunk(s) per job, "
                        + (f"jobs estimated above {long_ms:g} ms alone in a second lane" if long_ms > 0 else "one lane"),
            "arrival_rate_per_s": rate, "jobs_per_s": n_jobs / span, "factors_per_s": factors / span,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3), "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_latency_ms": float(lat.mean() * 1e3), "iterations": st["iterations"],
            "kmod_table_hits": st["kmod_hits"], "kmod_table_builds": st["kmod_builds"]}


def main():
    args = _args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as W
    import paper_2012_03771_amd as cs

    if args.mc_curve:
        torch.cuda.set_device(0)
        print(json.dumps(_mc_curve(cs, torch, W, np, args)), flush=True)
        return
    if args.scatter_table:
        torch.cuda.set_device(0)
        print(json.dumps({"metric": "scatter operations per second", "rows": _scatter_table(cs, torch)}), flush=True)
        return
    if args.table_a2:
        torch.cuda.set_device(0)
        print(json.dumps(_table_a2(cs, torch, W, [int(x) for x in args.a2_rows.split(",")])), flush=True)
        return
    job = W.SINGLE_JOBS[args.workload]
    scatter = {"auto": cs.SCATTER_AUTO, "atomic": cs.SCATTER_ATOMIC, "bytes": cs.SCATTER_BYTES,
               "list": cs.SCATTER_LIST}[args.scatter]
    tune = cs.Tune(large_mode=cs.LARGE_G if args.mode == "g" else cs.LARGE_THREE_GAP, scatter=scatter,
                   thr=int(args.thr_mult * (2 * job.sl + 1)))
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_probe:
        src = torch.ones(args.copy_probe * 2**20 // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    lay, bitmap, counts, ws = cs.binding.alloc_outputs(job, tune)
    print(f"# workload {args.workload} rows={lay.n_m} cols={lay.n_x} ws={lay.ws_bytes/2**30:.2f} GiB "
          f"thr={lay.thr}", file=sys.stderr, flush=True)

    def step():
        cs.sieve_into(job, bitmap, counts, ws, tune, stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"# warmup {i} done", file=sys.stderr, flush=True)
    ms_per_step = None
    if not args.phase_only:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms_per_step = (t1 - t0) * 1e3 / args.steps
        print(f"# {args.steps} steps: {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)
    diag = cs.diag_read(ws, stream)
    factors = int(counts.to(torch.int64).sum().item())
    ref_bitmap = bitmap.clone()
    ref_counts = counts.clone()

    # phase timing with HIP events on the launch stream: prepare, small branch, large branch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    bitmap.zero_()
    counts.zero_()
    ev[0].record(stream)
    cs.prepare(job, ws, tune, stream)
    ev[1].record(stream)
    ts = cs.Tune(**{**tune.__dict__, "branches": cs.BRANCH_SMALL})
    cs.sieve_range(job, 2, job.limit, bitmap, counts, ws, ts, stream)
    ev[2].record(stream)
    tl = cs.Tune(**{**tune.__dict__, "branches": cs.BRANCH_LARGE})
    cs.sieve_range(job, 2, job.limit, bitmap, counts, ws, tl, stream)
    ev[3].record(stream)
    torch.cuda.synchronize()
    phases = {"prepare": ev[0].elapsed_time(ev[1]), "small": ev[1].elapsed_time(ev[2]),
              "large": ev[2].elapsed_time(ev[3])}
    same = bool(torch.equal(bitmap, ref_bitmap) and torch.equal(counts, ref_counts))
    diag_ph = cs.diag_read(ws, stream)
    if ms_per_step is None:
        ms_per_step = sum(phases.values())
    print(f"# phases ms {phases} identical={same}", file=sys.stderr, flush=True)

    T = ms_per_step / 1e3
    value = factors / T
    primes_per_s = diag.n_primes / T

    # roofline of the large branch (one k_large launch per step): algorithmic VALU operations
    # = units counted by the kernel x their operation prices (paper_2012_03771_amd/roofline.py),
    # over the kernel's own duration (HIP events around the launch, on its stream)
    from paper_2012_03771_amd import roofline as RL
    t_large = (diag_ph.large_kernel_ms or phases["large"]) / 1e3
    # a single job below 2^42 forms K mod p of its large primes in the kernel (cs_tune.kmod AUTO)
    groups = RL.kmod_groups(job.P, job.d) if max(job.limit, job.P) < 2**42 else 0
    ops = RL.large_branch_ops(diag_ph, args.mode == "three_gap", groups)
    roof = {"bound": "alu", "kernel": "k_large", "achieved": ops / t_large / 1e12, "peak": ALU_PEAK_OPS / 1e12,
            "unit": "Tops/s (VALU lane-ops)", "frac": ops / t_large / ALU_PEAK_OPS,
            "traffic": args.traffic_gb if args.traffic_gb is not None else _kernel_traffic(args.mode),
            "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
            "traffic_source": "committed rocprofv3 counter profile of this kernel source (profiles/traffic.json), "
                              "not measured by this run; null when the sources changed since",
            "ops_per_launch": ops, "op_units": {"g_levels": diag_ph.g_levels, "g_calls": diag_ph.g_calls,
                                                "raw_hits": diag_ph.large_raw_hits,
                                                "large_primes": diag_ph.large_primes,
                                                "kmod_groups_formed": groups},
            "launch_ms": t_large * 1e3, "large_phase_ms": phases["large"],
            "valu_issue_frac": _valu_issue(args.mode),
            "valu_issue_source": "committed rocprofv3 SQ_INSTS_VALU profile (profiles/traffic.json), not measured by "
                                 "this run: x 4 cycles / (1024 SIMDs x 2.4 GHz x launch time)"}
    if roof["traffic"] is not None:
        # the same launch against the HBM roofline: measured bytes over the launch time
        roof["hbm_achieved_gb_s"] = roof["traffic"] / t_large
        roof["hbm_frac"] = roof["traffic"] * 1e9 / t_large / HBM_PEAK
    if lay.scatter == cs.SCATTER_BYTES and not args.no_atomic_probe:
        # the hits are device-scope atomic adds into byte counters: their rate against the rate of
        # the same atomics at random words of a buffer of the same size
        n_words = lay.n_m * lay.row_words * 8
        rate = _scatter_probe(cs, torch, n_words, 1 << 28)
        hits = diag_ph.large_hits
        roof["atomics"] = {"count": hits, "achieved_per_s": hits / t_large, "probe_per_s": rate,
                           "frac": hits / t_large / rate,
                           "probe": f"cs_probe_scatter: 2^28 device-scope atomic adds at hashed random words of "
                                    f"{n_words * 4 / 2**30:.2f} GiB (the byte counters' size), indices in registers"}
        print(f"# atomics: {hits / t_large:.3e}/s in k_large, probe {rate:.3e}/s", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": value, "unit": "factors/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": args.workload, "P": job.P, "d": job.d, "m_start": job.m_start,
                   "m_inc": job.m_inc, "sl": job.sl, "limit": job.limit, "rows": lay.n_m, "cols": lay.n_x,
                   "large_mode": args.mode, "thr": lay.thr},
        "primes_per_s": primes_per_s, "factors": factors, "n_primes": diag.n_primes,
        "phases_ms": phases, "phases_identical": same,
        "diag": {k: getattr(diag_ph, k) for k in ("small_pairs", "small_marks", "large_raw_hits", "large_hits",
                                                  "g_calls", "g_levels")},
        "roofline": roof,
    }
    if args.prp_rows > 0:
        print(f"# prp leg on {min(args.prp_rows, lay.n_m)} rows ...", file=sys.stderr, flush=True)
        out["prp"] = _prp_leg(cs, torch, np, job, bitmap, min(args.prp_rows, lay.n_m), stream)
        print(f"# prp {out['prp']['s']:.3f} s, {out['prp']['tests_per_s']:.3e} tests/s, "
              f"frac {out['prp']['roofline']['frac']:.3f}", file=sys.stderr, flush=True)
    if not args.no_g and args.mode != "g":
        tg = cs.Tune(large_mode=cs.LARGE_G)
        ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        bitmap.zero_()
        counts.zero_()
        ev2[0].record(stream)
        cs.prepare(job, ws, tg, stream)
        ev2[1].record(stream)
        cs.sieve_range(job, 2, job.limit, bitmap, counts, ws, cs.Tune(large_mode=cs.LARGE_G, branches=cs.BRANCH_SMALL), stream)
        ev2[2].record(stream)
        cs.sieve_range(job, 2, job.limit, bitmap, counts, ws, cs.Tune(large_mode=cs.LARGE_G, branches=cs.BRANCH_LARGE), stream)
        ev2[3].record(stream)
        torch.cuda.synchronize()
        dg = cs.diag_read(ws, stream)
        ph = {"prepare": ev2[0].elapsed_time(ev2[1]), "small": ev2[1].elapsed_time(ev2[2]),
              "large": ev2[2].elapsed_time(ev2[3])}
        og = RL.large_branch_ops(dg, False, groups)
        tlg = (dg.large_kernel_ms or ph["large"]) / 1e3
        out["g_mode"] = {"phases_ms": ph, "ms_per_step": sum(ph.values()), "thr": cs.plan(job, tg).thr,
                         "factors_per_s": factors / (sum(ph.values()) / 1e3),
                         "identical": bool(torch.equal(bitmap, ref_bitmap) and torch.equal(counts, ref_counts)),
                         "g_calls": dg.g_calls, "g_levels": dg.g_levels,
                         "roofline": {"bound": "alu", "kernel": "k_large", "achieved": og / tlg / 1e12,
                                      "peak": ALU_PEAK_OPS / 1e12, "unit": "Tops/s (VALU lane-ops)",
                                      "frac": og / tlg / ALU_PEAK_OPS, "ops_per_launch": og,
                                      "op_units": {"g_levels": dg.g_levels, "g_calls": dg.g_calls,
                                                   "raw_hits": dg.large_raw_hits, "large_primes": dg.large_primes},
                                      "traffic": _kernel_traffic("g"), "valu_issue_frac": _valu_issue("g"),
                                      "traffic_source": "committed profile (profiles/traffic.json), not this run",
                                      "launch_ms": tlg * 1e3, "large_phase_ms": ph["large"]}}
    mode_b = cs.LARGE_G if args.mode == "g" else cs.LARGE_THREE_GAP
    gpu_counts = ref_counts.cpu().numpy().view(np.uint32).copy()
    del bitmap, counts, ws, ref_bitmap, ref_counts
    torch.cuda.empty_cache()
    if not args.no_batch:
        print("# batch leg ...", file=sys.stderr, flush=True)
        out["batch"] = _batch_leg(cs, torch, W, mode_b, autotune=not args.no_autotune)
        print(f"# batch {out['batch']['ms_batched']:.1f} ms vs sequential {out['batch']['ms_sequential']:.1f} ms",
              file=sys.stderr, flush=True)
    if not args.no_serve:
        print("# serve capacity ...", file=sys.stderr, flush=True)
        cap = _server_capacity(cs, W, mode_b, chunks=args.serve_chunks, long_ms=args.serve_long_ms)
        loads = sorted({float(x) for x in args.serve_loads.split(",")} | {0.8})
        curve = []
        for load in loads:
            rate = load * cap
            print(f"# serve leg at {rate:.1f} jobs/s ({load} of capacity {cap:.1f}) ...", file=sys.stderr, flush=True)
            leg = _serve_leg(cs, torch, W, mode_b, rate, args.serve_jobs, args.serve_warmup, args.serve_chunks,
                             args.serve_long_ms)
            leg["load"] = load
            leg["capacity_jobs_per_s"] = cap
            print(f"# serve {load}: p50 {leg['p50_latency_ms']:.1f} ms p99 {leg['p99_latency_ms']:.1f} ms",
                  file=sys.stderr, flush=True)
            if load == 0.8:
                out["serve"] = leg
            curve.append({k: leg[k] for k in ("load", "arrival_rate_per_s", "jobs_per_s", "p50_latency_ms",
                                             "p99_latency_ms", "mean_latency_ms", "iterations")})
        out["serve"]["curve"] = curve
        out["serve"]["alone"] = _alone_times(cs, torch, W, mode_b, 256)
        print(f"# served jobs alone: p50 {out['serve']['alone']['p50_ms']:.2f} ms p99 "
              f"{out['serve']['alone']['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    if not args.no_cpu:
        print("# cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = _cpu_baseline(job, args.cpu_rows, gpu_counts)
        print(f"# cpu baseline {out['cpu_baseline']['value']:.3e} factors/s on {out['cpu_baseline']['cores']} "
              f"threads, rows equal: {out['cpu_baseline'].get('rows_equal_gpu')}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

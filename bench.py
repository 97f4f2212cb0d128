"""Benchmark of the Combined Sieve hot path on one MI355X.

A step is one whole cs_sieve call on the paper-scale job 953#/210, m in [1e8, 1e8 + 1e6),
sl = 20000, primes up to 1e10: prime table, K mod p for all 455,052,511 primes, row/column
maps, the small-prime branch and the large-prime branch, with every input built on the device
inside the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
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


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", choices=["g", "three_gap"], default="g")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--cpu-rows", type=int, default=16)
    ap.add_argument("--cpu-pmax", type=int, default=2**30)
    ap.add_argument("--workload", default="paper_953")
    ap.add_argument("--phase-only", action="store_true", help="time the phases once, no steps")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of this many MiB (a known-size reference for "
                         "HBM byte counters)")
    return ap.parse_args()


def _cpu_baseline(job, n_rows, p_max):
    """The oracle as it stands (plain per-interval sieve, bignum N mod p for every row and
    prime) on a bounded sample: n_rows rows of the job and the primes <= p_max."""
    import numpy as np
    import workloads as W
    from oracle import coracle
    import paper_2012_03771_amd as cs
    lay = cs.plan(job)
    rec = W.RECORD_GAPS[0]
    must = []
    if (job.P, job.d) == (rec[0], rec[1]) and job.m_start <= rec[2] < job.m_start + job.m_inc:
        ms_all = cs.rows(job)
        must = [int(np.searchsorted(ms_all, rec[2]))]
        rows = W.sample_rows(lay.n_m, n_rows, seed=11, must=must)
        ms = ms_all[rows]
    else:
        ms_all = cs.rows(job)
        rows = W.sample_rows(lay.n_m, n_rows, seed=11)
        ms = ms_all[rows]
    threads = len(os.sched_getaffinity(0))
    threads = min(threads, 16)
    t0 = time.perf_counter()
    _, counts = coracle.sieve_rows(job.P, job.d, job.sl, ms, 2, min(p_max, job.limit),
                                   mode=coracle.DIRECT, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": float(counts.sum()) / dt, "unit": "factors/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(ms)} rows of {lay.n_m} (first, last, record-gap row, seeded), primes <= "
                      f"{min(p_max, job.limit)}, plain per-interval sieve with bignum N mod p "
                      f"(direct mode), {dt:.1f} s wall"}


def main():
    args = _args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as W
    import paper_2012_03771_amd as cs

    job = W.SINGLE_JOBS[args.workload]
    tune = cs.Tune(large_mode=cs.LARGE_G if args.mode == "g" else cs.LARGE_THREE_GAP)
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

    # roofline of the large branch (one k_large launch per step): algorithmic VALU operations =
    # recursion levels x operations per level + solves x per-solve operations
    from paper_2012_03771_amd import roofline as RL
    t_large = phases["large"] / 1e3
    ops = RL.large_branch_ops(diag_ph)
    roof = {"bound": "alu", "kernel": "k_large", "achieved": ops / t_large / 1e12, "peak": ALU_PEAK_OPS / 1e12,
            "unit": "Tops/s (VALU lane-ops)", "frac": ops / t_large / ALU_PEAK_OPS, "traffic": None,
            "ops_per_launch": ops, "launch_ms": phases["large"]}

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
    if not args.no_cpu:
        print("# cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = _cpu_baseline(job, args.cpu_rows, args.cpu_pmax)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Autotuner for the sieve's launch knobs, per job-shape bucket.

A bucket is (log2 rows, log2 columns, half-decade of the sieve limit, d).  For the first job of
a bucket every candidate tuning is timed with cs_sieve (one warm-up, then the fastest of two
timed runs, HIP events on the launch stream) and the fastest is kept for the whole bucket.
Candidates vary the small/large threshold (a multiple of S = 2 sl + 1, Section 5's C_mult) and
the expected hits per large-branch work item; all give identical outputs, so the choice only
affects speed.

tune_batch then tunes the whole batch: the batch path (one persistent launch over a device task
queue, or per-job launches over lane streams) and the rows per small-branch LDS tile (the
m-window of a tile), timing each combination on the batch itself replayed from its hipGraph, and
then the per-job thresholds against one rule for jobs that share the device (44 n_x).
"""
from __future__ import annotations

import json
import math
import os

from . import binding as B

DEFAULT_CANDIDATES = [
    {"thr_mult": m, "hits_per_item": h, "large_mode": B.LARGE_THREE_GAP}
    for m in (8, 20, 40) for h in (512, 2048)
]


class Autotuner:
    def __init__(self, candidates=None, cache_path: str | None = None):
        self.candidates = candidates or DEFAULT_CANDIDATES
        self.cache_path = cache_path
        self.cache: dict[str, dict] = {}
        self.timings: dict[str, list] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    @staticmethod
    def bucket(job) -> str:
        lay = B.plan(job)
        P, d, m_start, m_inc, sl, limit = B.job_tuple(job)
        return "%d/%d/%.1f/%d" % (round(math.log2(max(lay.n_m, 1))), round(math.log2(max(lay.n_x, 1))),
                                  round(2 * math.log10(limit)) / 2, d)

    @staticmethod
    def _tune_of(job, cand) -> B.Tune:
        sl = B.job_tuple(job)[4]
        return B.Tune(thr=int(cand["thr_mult"] * (2 * sl + 1)), hits_per_item=cand["hits_per_item"],
                      large_mode=cand["large_mode"])

    def _time(self, job, tune, bitmap, counts, ws) -> float:
        import torch
        s = torch.cuda.current_stream()
        B.sieve_into(job, bitmap, counts, ws, tune, s)
        best = float("inf")
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            B.sieve_into(job, bitmap, counts, ws, tune, s)
            e1.record(s)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    def tune(self, job) -> B.Tune:
        key = self.bucket(job)
        if key not in self.cache:
            import torch
            lays = [B.plan(job, self._tune_of(job, c)) for c in self.candidates]
            lay0 = lays[0]
            bitmap = torch.empty((lay0.n_m, lay0.row_words), dtype=torch.int32, device="cuda")
            counts = torch.empty((lay0.n_m,), dtype=torch.int32, device="cuda")
            ws = torch.empty((max(L.ws_bytes for L in lays),), dtype=torch.uint8, device="cuda")
            times = [self._time(job, self._tune_of(job, c), bitmap, counts, ws) for c in self.candidates]
            best = min(range(len(times)), key=times.__getitem__)
            self.cache[key] = dict(self.candidates[best])
            self.timings[key] = times
            del bitmap, counts, ws
            if self.cache_path:
                with open(self.cache_path, "w") as f:
                    json.dump(self.cache, f, indent=1)
        return self._tune_of(job, self.cache[key])

    def tune_all(self, jobs):
        return [self.tune(j) for j in jobs]

    # batch-level candidates: the persistent kernel with 256 to 4,096 large-branch items (primes x
    # m-chunks) per task and 8 or 16 rows per small-branch tile, and the lane path
    BATCH_CANDIDATES = ([{"path": B.BATCH_PERSISTENT, "items_per_task": ipt, "tile_rows": rows}
                         for ipt, rows in ((256, 16), (1024, 8), (1024, 16), (4096, 16))]
                        + [{"path": B.BATCH_LANES, "items_per_task": 0, "tile_rows": rows} for rows in (8, 16)])

    # threshold per column of the interval for jobs that share the device (the small and large
    # branches of many jobs then add up rather than overlap: n_m 1.25 ps per small prime against
    # n_m n_x / p hit atomics of 55 ps per large one, least at thr = 44 n_x)
    THR_PER_COLUMN = 44

    def tune_batch(self, jobs, reps: int = 2):
        """Per-job tunings (tune_all), then the batch path, items per task and small-branch tile
        rows that run the whole batch fastest; for that combination, the per-job thresholds are
        then set against thr = 44 n_x for every job, and the faster kept.  Returns (tunes, batch
        options, timings)."""
        import dataclasses
        import time
        import torch
        base = self.tune_all(jobs)
        timings = []
        best = None

        def timed(tunes, cand):
            try:
                batch = B.Batch(jobs, tunes, path=cand["path"], items_per_task=cand["items_per_task"])
            except B.CsError:
                return None                               # this path does not admit the jobs
            bm, ct = batch.alloc_outputs()
            batch.run(bm, ct, use_graph=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                batch.run(bm, ct, use_graph=True)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
            batch.close()
            del bm, ct
            return t

        for cand in self.BATCH_CANDIDATES:
            tunes = [dataclasses.replace(t, tile_rows=cand["tile_rows"]) for t in base]
            t = timed(tunes, cand)
            if t is None:
                continue
            timings.append({**cand, "thr": "per job", "ms": t * 1e3})
            if best is None or t < best[0]:
                best = (t, cand, tunes)
        cand = best[1]
        tunes = [dataclasses.replace(t, tile_rows=cand["tile_rows"], large_mode=B.LARGE_THREE_GAP,
                                     thr=self.THR_PER_COLUMN * max(1, B.plan(j).n_x))
                 for t, j in zip(base, jobs)]
        t = timed(tunes, cand)
        if t is not None:
            timings.append({**cand, "thr": "%d n_x" % self.THR_PER_COLUMN, "ms": t * 1e3})
            if t < best[0]:
                best = (t, cand, tunes)
        torch.cuda.empty_cache()
        return best[2], {"path": best[1]["path"], "items_per_task": best[1]["items_per_task"]}, timings

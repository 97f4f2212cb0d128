// Batched sieving: many jobs with different P, d, m ranges, intervals and limits in one
// sequence of fused launches, captured once in a hipGraph and replayed.
//
// The prime table is built once up to the largest limit and shared; every other table is per
// job.  The preparation kernels cover all jobs in one launch each: they take the job from
// blockIdx.y, and K mod p runs over the flattened prime index space of all jobs.  Each job's two
// sieve branches then run as single-job launches (LDS tables, uniform job fields) spread over
// lane streams forked from and joined back into the caller's stream inside the graph.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/csieve.h"
#include "batch_internal.h"
#include "device.h"
#include "launch.h"
#include "plan.h"

using namespace cs;

#define CS_TRY(expr)                                 \
  do {                                               \
    if ((expr) != hipSuccess) return CS_EDEVICE;     \
  } while (0)

namespace cs {

static uint64_t a256(uint64_t x) { return (x + 255) & ~255ull; }

void retile_small(Plan& pl, uint32_t lds_ct_words, int n_cu, const cs_tune* tune, uint32_t lds_budget) {
  const uint32_t ct_bytes = lds_ct_words * 8u;
  uint32_t rows = lds_budget > ct_bytes ? (lds_budget - ct_bytes) / (4u * pl.row_words + 8u) : 0u;
  rows = std::max(1u, std::min(rows, kTileRowsMax));
  if (tune && tune->tile_rows) rows = std::min(rows, tune->tile_rows);
  pl.tile_rows = rows;
  pl.n_windows = (uint32_t)((pl.n_m + rows - 1) / rows);
  pl.lds_ct_words = lds_ct_words;
  pl.lds_bytes = ct_bytes + 4u * rows * pl.row_words + 8u * rows;   // tile, counts, m offsets
  const double est_small = (double)pl.thr / std::max(1.0, log((double)pl.thr));
  uint32_t max_slices = (uint32_t)std::max(1.0, std::min(64.0, est_small / 512.0));
  uint32_t slices = pl.n_windows ? (uint32_t)((4u * (uint32_t)n_cu + pl.n_windows - 1) / pl.n_windows) : 1;
  slices = std::max(1u, std::min(slices, max_slices));
  if (tune && tune->small_slices) slices = std::min(tune->small_slices, 256u);
  pl.n_slices = slices;
  pl.small_blocks = (uint32_t)std::min<uint64_t>(std::max<uint64_t>((uint64_t)pl.n_windows * slices, 1), 1ull << 31);
}

cs_status multi_build(MultiJob& b, const cs_job* jobs, const cs_tune* tunes, uint32_t n, int n_cu,
                      uint64_t prime_extent, int want_persistent) {
  b.n = n;
  b.n_cu = n_cu;
  b.plans.assign(n, Plan());
  uint64_t Lp = std::max<uint64_t>(prime_extent, 2);
  uint32_t max_ct = 0;
  // byte counters for the large hits when every job with rows can use them (one kernel variant
  // serves all jobs of the fused launch), else the atomic scatter for all
  b.bytes = true;
  for (uint32_t pass = 0; pass < 2; ++pass) {
    for (uint32_t i = 0; i < n; ++i) {
      cs_status st = make_plan(&jobs[i], tunes ? &tunes[i] : nullptr, n_cu, &b.plans[i], false, true, b.bytes);
      if (st) return st;
    }
    bool all = true;
    for (uint32_t i = 0; i < n; ++i) all = all && (b.plans[i].n_m == 0 || b.plans[i].scatter_bytes);
    if (all || !b.bytes) break;
    b.bytes = false;
  }
  for (uint32_t i = 0; i < n; ++i) {
    Lp = std::max(Lp, b.plans[i].Lp);
    max_ct = std::max(max_ct, b.plans[i].ct_words);
  }
  b.max_rows = 0;
  for (uint32_t i = 0; i < n; ++i) b.max_rows = std::max<uint64_t>(b.max_rows, b.plans[i].n_m);
  if (Lp >= kWideLo) return CS_ERANGE;
  b.Lp = Lp;
  b.lds_ct_words = max_ct * 8u <= kLdsCtMax ? max_ct : 0u;
  // The persistent kernel needs one enumeration for all jobs and every job's column table (and
  // residue table of d) in LDS beside a small-branch tile of at least one row.
  {
    bool ok = b.lds_ct_words > 0;
    uint32_t max_dp = 0;
    b.large_mode = b.plans[0].large_mode;
    for (uint32_t i = 0; i < n && ok; ++i) {
      const Plan& pl = b.plans[i];
      ok = pl.large_mode == b.large_mode;
      max_dp = std::max<uint32_t>(max_dp, (uint32_t)pl.dpre.size());
      if (ok && pl.n_m > 0)
        ok = (uint64_t)b.lds_ct_words * 8u + 4ull * pl.row_words + 8u <= kPersistLds;
    }
    uint32_t large_lds = b.lds_ct_words * 8u + ((max_dp * 2u + 3u) & ~3u);
    // K's groups of the jobs that form K mod p in the large branch, after the tables, 8-aligned
    size_t max_kg = 0;
    for (uint32_t i = 0; i < n; ++i)
      if (b.plans[i].kmod_fused) max_kg = std::max(max_kg, std::max<size_t>(b.plans[i].kq.size(), 1));
    b.kg_off_words = 0;
    if (max_kg) {
      const uint32_t off = (large_lds + 7u) & ~7u;
      b.kg_off_words = off / 4u;
      large_lds = off + 8u * (uint32_t)max_kg;
    }
    ok = ok && large_lds <= kPersistLds;
    if (want_persistent > 0 && !ok) return CS_EINVAL;
    b.persistent = want_persistent != 0 && ok;
    b.persist_lds = large_lds;
  }
  b.units = 0;
  b.lds_bytes = 0;
  b.max_words = 0;
  b.max_m_inc = 0;
  b.max_sl = 0;
  b.kmod_cap = 0;
  for (uint32_t i = 0; i < n; ++i) {
    Plan& pl = b.plans[i];
    retile_small(pl, b.lds_ct_words, n_cu, tunes ? &tunes[i] : nullptr, b.persistent ? kPersistLds : kLdsBudget);
    if (pl.n_m > 0) b.lds_bytes = std::max(b.lds_bytes, pl.lds_bytes);   // jobs without rows launch nothing
    b.max_words = std::max<uint64_t>(b.max_words, pl.n_m * (uint64_t)pl.row_words);
    b.max_m_inc = std::max<uint64_t>(b.max_m_inc, pl.job.m_inc);
    b.max_sl = std::max(b.max_sl, pl.job.sl);
    b.kmod_cap += pl.kmod_fused ? std::min(pi_upper(pl.job.limit), pi_upper(pl.thr)) : pi_upper(pl.job.limit);
  }
  // device memory: shared prime table, job descriptors, prefix arrays, per-job tables
  b.n_seg = (Lp >> kSegLog) + 1;
  b.cap = pi_upper(Lp);
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) { uint64_t at = o; o = a256(o + std::max<uint64_t>(bytes, 8)); return at; };
  b.o_nbase = take(8);
  b.o_np = take(8);
  b.o_base = take(kBaseCap * 4ull);
  b.o_flags = take(b.n_seg * kSegWords * 4ull);
  b.o_cnt = take(b.n_seg * 4ull);
  b.o_off = take(b.n_seg * 8ull);
  b.o_primes = take(b.cap * 8ull);
  b.o_jobs = take(sizeof(JobDev) * (uint64_t)n);
  b.o_lim = take(8ull * (n + 1));
  b.o_items = take(8ull * (n + 1));
  b.o_tbase = take(8ull * (2ull * n + 1));
  b.o_next = take(8);
  b.persist_lds = std::max(b.persist_lds, b.lds_bytes);
  b.persist_blocks = (uint32_t)n_cu * kPersistBlocksPerCu;
  b.job_off.resize(n);
  for (uint32_t i = 0; i < n; ++i) b.job_off[i] = take(b.plans[i].ws.total);
  b.mem_bytes = o;
  return CS_OK;
}

cs_status multi_alloc(MultiJob& b, hipStream_t s) {
  uint8_t* mem = nullptr;
  if (hipMalloc(&mem, b.mem_bytes) != hipSuccess) return CS_ENOMEM;
  return multi_use_memory(b, mem, s);
}

cs_status multi_use_memory(MultiJob& b, uint8_t* mem, hipStream_t s) {
  b.mem = mem;
  uint8_t* m = b.mem;
  b.pw.n_base = reinterpret_cast<uint32_t*>(m + b.o_nbase);
  b.pw.n_primes = reinterpret_cast<uint64_t*>(m + b.o_np);
  b.pw.base = reinterpret_cast<uint32_t*>(m + b.o_base);
  b.pw.flags = reinterpret_cast<uint32_t*>(m + b.o_flags);
  b.pw.seg_count = reinterpret_cast<uint32_t*>(m + b.o_cnt);
  b.pw.seg_off = reinterpret_cast<uint64_t*>(m + b.o_off);
  b.pw.primes = reinterpret_cast<uint64_t*>(m + b.o_primes);
  b.pw.cap = b.cap;
  b.jobs_dev = reinterpret_cast<JobDev*>(m + b.o_jobs);
  b.lim_base = reinterpret_cast<uint64_t*>(m + b.o_lim);
  b.items_base = reinterpret_cast<uint64_t*>(m + b.o_items);
  b.tbase = reinterpret_cast<uint64_t*>(m + b.o_tbase);
  b.task_next = reinterpret_cast<unsigned long long*>(m + b.o_next);
  b.jds.resize(b.n);
  uint64_t unit_base = 0;
  for (uint32_t i = 0; i < b.n; ++i) {
    const Plan& pl = b.plans[i];
    uint8_t* ws = m + b.job_off[i];
    b.jds[i] = make_jobdev(pl, ws, b.pw.primes, b.pw.n_primes);
    if (pl.scatter_bytes)   // the counters start cleared; every run's fold clears them again
      CS_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(ws + pl.ws.hitbytes), pl.n_m * (uint64_t)pl.row_words * 8ull, 0u, s));
    b.jds[i].small_unit_base = 0;             // each job's small branch is its own launch
    b.jds[i].prime_cap = b.cap;
    // in the persistent kernel a job's small units run beside its large items: with the atomic
    // scatter both OR into the bitmap, so the small tiles merge with atomics
    if (b.persistent && !pl.scatter_bytes) b.jds[i].small_atomic = 1;
    unit_base += (uint64_t)pl.n_windows * pl.n_slices;
    if (!pl.dpre.empty()) {
      CS_TRY(launch_upload(ws + pl.ws.dpre, pl.dpre.data(), pl.dpre.size() * 2ull, s));
      CS_TRY(launch_upload(ws + pl.ws.dres, pl.dres.data(), pl.dres.size() * 2ull, s));
    }
    if (pl.dpat_on) {
      b.max_phi = std::max(b.max_phi, pl.phi_d);
      b.max_rw = std::max(b.max_rw, pl.row_words);
    }
  }
  b.units = unit_base;
  return CS_OK;
}

cs_status multi_bind(MultiJob& b, uint32_t* const* bitmaps, uint32_t* const* counts, hipStream_t s) {
  for (uint32_t i = 0; i < b.n; ++i) {
    if (b.plans[i].n_m > 0 && (!bitmaps[i] || !counts[i])) return CS_EINVAL;
    b.jds[i].bitmap = bitmaps[i];
    b.jds[i].counts = counts[i];
    CS_TRY(launch_write_job(b.jds[i], b.jobs_dev + i, s));
  }
  return CS_OK;
}

// The whole sieve of every job: outputs cleared, shared prime table, per-job tables, both
// branches over all primes <= each job's limit.
cs_status multi_enqueue(MultiJob& b, hipStream_t s) {
  const uint32_t n = b.n;
  CS_TRY(launch_fill_jobs(b.jobs_dev, n, b.max_words, s));
  CS_TRY(launch_zero_ctrls(b.jobs_dev, n, s));
  CS_TRY(launch_primes(b.Lp, b.pw, s));
  CS_TRY(launch_prep_tables(b.jobs_dev, n, s));
  CS_TRY(launch_kmod(b.jobs_dev, n, b.lim_base, b.kmod_cap, b.n_cu, s));
  CS_TRY(launch_rows_cols(b.jobs_dev, n, b.max_m_inc, b.max_sl, b.n_cu, s));
  CS_TRY(launch_dpattern(b.jobs_dev, n, b.max_phi, b.max_rw, s));
  CS_TRY(launch_prep_bounds(b.jobs_dev, n, s));
  if (b.persistent) {
    // every job's small units and large items in one launch, then the byte counters' fold
    CS_TRY(launch_batch_persistent(b.jobs_dev, n, b.tbase, b.task_next, b.persist_blocks, b.persist_lds,
                                   b.lds_ct_words, b.kg_off_words, b.bytes ? 1u : 0u, b.large_mode, b.items_per_task,
                                   b.order, s));
    if (b.bytes) CS_TRY(launch_fold_bytes(b.jobs_dev, n, b.max_rows, b.n_cu, s));
    return CS_OK;
  }
  // Each job's branches as single-job launches (LDS tables, uniform job fields, byte counters),
  // jobs spread over the lanes so several run at once (on s in turn when there are no lanes).
  const uint32_t nl = (uint32_t)b.lanes.size();
  if (nl) {
    CS_TRY(hipEventRecord(b.ev_fork, s));
    for (uint32_t l = 0; l < nl; ++l) CS_TRY(hipStreamWaitEvent(b.lanes[l], b.ev_fork, 0));
  }
  for (uint32_t i = 0; i < n; ++i) {
    const Plan& pl = b.plans[i];
    if (pl.n_m == 0) continue;
    hipStream_t ls = nl ? b.lanes[i % nl] : s;
    const JobDev* jd = b.jobs_dev + i;
    uint64_t* ib = reinterpret_cast<uint64_t*>(b.mem + b.job_off[i] + pl.ws.items_base);
    CS_TRY(launch_items_scan(jd, 1, ib, ls));
    const uint64_t units = (uint64_t)pl.n_windows * pl.n_slices;
    CS_TRY(launch_small(jd, 1, units, pl.lds_bytes, pl.lds_ct_words, pl.small_blocks, ls, pl.small_hit_rows));
    CS_TRY(launch_large(jd, 1, ib, b.jds[i].ctrl->diag, &b.jds[i].ctrl->dec[0][0], pl.large_blocks, pl.large_lds_bytes, pl.large_lds_ct_words,
                        (uint32_t)pl.dpre.size(), pl.scatter_bytes ? 1u : 0u, pl.large_mode, ls));
    if (pl.scatter_bytes) CS_TRY(launch_fold_bytes(jd, 1, pl.n_m, b.n_cu, ls));
  }
  for (uint32_t l = 0; l < nl; ++l) {
    CS_TRY(hipEventRecord(b.ev_done[l], b.lanes[l]));
    CS_TRY(hipStreamWaitEvent(s, b.ev_done[l], 0));
  }
  return CS_OK;
}

cs_status batch_opts_of(const cs_batch_opts* opts, int* want_persistent) {
  const uint32_t path = opts ? opts->path : CS_BATCH_AUTO;
  if (path > CS_BATCH_LANES) return CS_EINVAL;
  if (opts && (opts->items_per_task % 256u || opts->items_per_task > 8192u || opts->blocks_per_cu > 8u ||
               opts->order > CS_ORDER_BY_JOB))
    return CS_EINVAL;
  *want_persistent = path == CS_BATCH_PERSISTENT ? 1 : (path == CS_BATCH_LANES ? 0 : -1);
  return CS_OK;
}

// Defaults measured on the 64-job mixed batch (three-gap, autotuned jobs): 1,024 items per task in
// job order 249 ms, large tasks first 260 ms, 256 items per task 264-274 ms; the lane path 259 ms.
void apply_batch_opts(MultiJob& b, const cs_batch_opts* opts) {
  b.items_per_task = opts && opts->items_per_task ? opts->items_per_task : 1024u;
  const uint32_t order = opts ? opts->order : CS_ORDER_AUTO;
  b.order = order == CS_ORDER_LARGE_FIRST ? 0u : (order == CS_ORDER_SMALL_FIRST ? 1u : 2u);   // k_batch_queue's
  if (opts && opts->blocks_per_cu) b.persist_blocks = (uint32_t)b.n_cu * opts->blocks_per_cu;
}

cs_status multi_diag(const MultiJob& b, cs_diag* out) {
  memset(out, 0, sizeof(*out));
  uint64_t err = 0;
  for (uint32_t i = 0; i < b.n; ++i) {
    JobCtrl c;
    if (hipMemcpy(&c, b.jds[i].ctrl, sizeof(JobCtrl), hipMemcpyDeviceToHost) != hipSuccess) return CS_EDEVICE;
    if (i == 0) out->n_primes = c.diag[D_NPRIMES];
    out->small_pairs += c.diag[D_SMALL_PAIRS];
    out->small_marks += c.diag[D_SMALL_MARKS];
    out->large_raw_hits += c.diag[D_LARGE_RAW];
    out->large_hits += c.diag[D_LARGE_HITS];
    out->g_calls += c.diag[D_G_CALLS];
    out->g_levels += c.diag[D_G_LEVELS];
    err |= c.diag[D_ERROR];
    out->small_primes += c.diag[D_SMALL_PRIMES];
    out->large_primes += c.diag[D_LARGE_PRIMES];
    for (int k = 0; k < kDecades; ++k) {
      out->dec_primes[k] += c.dec[DC_PRIMES][k];
      out->dec_raw_hits[k] += c.dec[DC_RAW][k];
      out->dec_hits[k] += c.dec[DC_HITS][k];
      out->dec_solves[k] += c.dec[DC_SOLVES][k];
      out->dec_levels[k] += c.dec[DC_LEVELS][k];
    }
    err |= c.error;
  }
  out->error_flags = err;
  return err ? CS_EDEVICE : CS_OK;
}

}  // namespace cs

struct cs_batch {
  MultiJob mj;
  int device = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uint32_t*> bound_b, bound_c;
  bool bound = false;
};

static cs_status create_lanes(MultiJob& m, uint32_t n) {
  if (hipEventCreateWithFlags(&m.ev_fork, hipEventDisableTiming) != hipSuccess) return CS_EDEVICE;
  for (uint32_t l = 0; l < n; ++l) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return CS_EDEVICE;
    m.lanes.push_back(st);
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return CS_EDEVICE;
    m.ev_done.push_back(ev);
  }
  return CS_OK;
}

static void destroy_lanes(MultiJob& m) {
  for (hipStream_t st : m.lanes) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipEvent_t ev : m.ev_done) (void)hipEventDestroy(ev);
  if (m.ev_fork) (void)hipEventDestroy(m.ev_fork);
  m.lanes.clear();
  m.ev_done.clear();
  m.ev_fork = nullptr;
}

static void drop_graph(cs_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

extern "C" cs_status cs_batch_create_ex(const cs_job* jobs, uint32_t n, const cs_tune* tunes,
                                        const cs_batch_opts* opts, cs_batch** out) {
  if (!jobs || !out || n == 0) return CS_EINVAL;
  *out = nullptr;
  int want = -1;
  cs_status st = batch_opts_of(opts, &want);
  if (st) return st;
  cs_batch* b = new (std::nothrow) cs_batch();
  if (!b) return CS_ENOMEM;
  if (hipGetDevice(&b->device) != hipSuccess) { delete b; return CS_EDEVICE; }
  st = multi_build(b->mj, jobs, tunes, n, device_cu_count(), 2, want);
  if (st) { delete b; return st; }
  apply_batch_opts(b->mj, opts);
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) { delete b; return CS_EDEVICE; }
  if (!b->mj.persistent && create_lanes(b->mj, std::min<uint32_t>(kBatchLanes, n)) != CS_OK) {
    (void)hipStreamDestroy(b->cap_stream);
    destroy_lanes(b->mj);
    delete b;
    return CS_EDEVICE;
  }
  st = multi_alloc(b->mj, b->cap_stream);
  if (st == CS_OK && hipStreamSynchronize(b->cap_stream) != hipSuccess) st = CS_EDEVICE;
  if (st) {
    if (b->mj.mem) (void)hipFree(b->mj.mem);
    (void)hipStreamDestroy(b->cap_stream);
    destroy_lanes(b->mj);
    delete b;
    return st;
  }
  *out = b;
  return CS_OK;
}

extern "C" cs_status cs_batch_create(const cs_job* jobs, uint32_t n, const cs_tune* tunes, cs_batch** out) {
  return cs_batch_create_ex(jobs, n, tunes, nullptr, out);
}

extern "C" uint32_t cs_batch_path(const cs_batch* b) {
  if (!b) return 0;
  return b->mj.persistent ? CS_BATCH_PERSISTENT : CS_BATCH_LANES;
}

extern "C" cs_status cs_batch_layout(const cs_batch* b, uint32_t i, cs_layout* out) {
  if (!b || !out || i >= b->mj.n) return CS_EINVAL;
  const Plan& pl = b->mj.plans[i];
  out->n_m = pl.n_m;
  out->n_x = pl.n_x;
  out->row_words = pl.row_words;
  out->bitmap_bytes = pl.n_m * (uint64_t)pl.row_words * 4ull;
  out->counts_bytes = pl.n_m * 4ull;
  out->ws_bytes = b->mj.mem_bytes;
  out->prime_cap = b->mj.cap;
  out->thr = pl.thr;
  out->scatter = pl.scatter_bytes ? CS_SCATTER_BYTES : CS_SCATTER_ATOMIC;
  out->reserved = 0;
  return CS_OK;
}

extern "C" cs_status cs_batch_run(cs_batch* b, uint32_t* const* d_bitmaps, uint32_t* const* d_counts,
                                  int use_graph, void* stream) {
  if (!b || !d_bitmaps || !d_counts) return CS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const uint32_t n = b->mj.n;
  bool same = b->bound;
  for (uint32_t i = 0; same && i < n; ++i) same = b->bound_b[i] == d_bitmaps[i] && b->bound_c[i] == d_counts[i];
  if (!same) {
    drop_graph(b);
    cs_status st = multi_bind(b->mj, d_bitmaps, d_counts, b->cap_stream);
    if (st) return st;
    if (hipStreamSynchronize(b->cap_stream) != hipSuccess) return CS_EDEVICE;
    b->bound_b.assign(d_bitmaps, d_bitmaps + n);
    b->bound_c.assign(d_counts, d_counts + n);
    b->bound = true;
  }
  if (!use_graph) return multi_enqueue(b->mj, s);
  if (!b->exec) {
    if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return CS_EDEVICE;
    cs_status st = multi_enqueue(b->mj, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (st || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return st ? st : CS_EDEVICE;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
      drop_graph(b);
      return CS_EDEVICE;
    }
  }
  CS_TRY(hipGraphLaunch(b->exec, s));
  return CS_OK;
}

extern "C" cs_status cs_batch_diag(cs_batch* b, cs_diag* out, void* stream) {
  if (!b || !out) return CS_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return CS_EDEVICE;
  return multi_diag(b->mj, out);
}

extern "C" cs_status cs_batch_destroy(cs_batch* b) {
  if (!b) return CS_OK;
  drop_graph(b);
  if (b->cap_stream) {
    (void)hipStreamSynchronize(b->cap_stream);
    (void)hipStreamDestroy(b->cap_stream);
  }
  destroy_lanes(b->mj);
  if (b->mj.mem) {
    (void)hipDeviceSynchronize();
    (void)hipFree(b->mj.mem);
  }
  delete b;
  return CS_OK;
}

// ---------------------------------------------------------------------------------------------
// One call: the whole batch on the caller's stream with a caller-provided workspace.
// ---------------------------------------------------------------------------------------------
extern "C" cs_status cs_batch_ws(const cs_job* jobs, uint32_t n, const cs_tune* tunes, uint64_t* ws_bytes) {
  if (!jobs || n == 0 || !ws_bytes) return CS_EINVAL;
  MultiJob mj;
  cs_status st = multi_build(mj, jobs, tunes, n, device_cu_count(), 2, -1);
  if (st) return st;
  *ws_bytes = mj.mem_bytes;
  return CS_OK;
}

extern "C" cs_status cs_sieve_batch(const cs_job* jobs, uint32_t n, const cs_tune* tunes, const cs_batch_opts* opts,
                                    uint32_t* const* d_bitmaps, uint32_t* const* d_counts, void* d_ws,
                                    uint64_t ws_bytes, void* stream) {
  if (!jobs || n == 0 || !d_bitmaps || !d_counts || !d_ws) return CS_EINVAL;
  int want = -1;
  cs_status st = batch_opts_of(opts, &want);
  if (st) return st;
  MultiJob mj;
  st = multi_build(mj, jobs, tunes, n, device_cu_count(), 2, want);
  if (st) return st;
  apply_batch_opts(mj, opts);
  if (ws_bytes < mj.mem_bytes) return CS_ERANGE;
  for (uint32_t i = 0; i < n; ++i)
    if (mj.plans[i].n_m > 0 && (!d_bitmaps[i] || !d_counts[i])) return CS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  st = multi_use_memory(mj, static_cast<uint8_t*>(d_ws), s);
  if (st) return st;
  st = multi_bind(mj, d_bitmaps, d_counts, s);
  if (st) return st;
  return multi_enqueue(mj, s);
}

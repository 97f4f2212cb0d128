// C ABI of the Combined Sieve library (declared in include/csieve.h).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/csieve.h"
#include "device.h"
#include "launch.h"
#include "plan.h"

using namespace cs;

#define CS_TRY(expr)                          \
  do {                                        \
    if ((expr) != hipSuccess) return CS_EDEVICE; \
  } while (0)

extern "C" const char* cs_strerror(cs_status st) {
  switch (st) {
    case CS_OK: return "ok";
    case CS_EINVAL: return "invalid argument";
    case CS_ERANGE: return "size out of range or buffer too small";
    case CS_ENOMEM: return "out of memory";
    case CS_EDEVICE: return "device error";
    case CS_EBUSY: return "busy";
    default: return "unknown status";
  }
}

extern "C" const char* cs_last_error(void) { return last_error_detail(); }

namespace {
void fill_layout(const Plan& pl, cs_layout* out) {
  out->n_m = pl.n_m;
  out->n_x = pl.n_x;
  out->row_words = pl.row_words;
  out->bitmap_bytes = pl.n_m * (uint64_t)pl.row_words * 4ull;
  out->counts_bytes = pl.n_m * 4ull;
  out->ws_bytes = pl.ws.total;
  out->prime_cap = pl.cap;
  out->thr = pl.thr;
  out->scatter = pl.scatter_list ? CS_SCATTER_LIST : (pl.scatter_bytes ? CS_SCATTER_BYTES : CS_SCATTER_ATOMIC);
  out->reserved = 0;
}
}  // namespace

extern "C" cs_status cs_plan(const cs_job* job, const cs_tune* tune, cs_layout* out) {
  if (!job || !out) return CS_EINVAL;
  Plan pl;
  cs_status st = make_plan(job, tune, 256, &pl);
  if (st) return st;
  fill_layout(pl, out);
  return CS_OK;
}

extern "C" cs_status cs_plan_chunked(const cs_job* job, const cs_tune* tune, uint64_t span, cs_layout* out) {
  if (!job || !out || !span) return CS_EINVAL;
  Plan pl;
  cs_status st = make_plan(job, tune, 256, &pl, true, true, true, span);
  if (st) return st;
  fill_layout(pl, out);
  return CS_OK;
}

extern "C" cs_status cs_columns(const cs_job* job, int32_t* x_of_col, uint64_t cap) {
  Plan pl;
  cs_status st = make_plan(job, nullptr, 256, &pl);
  if (st) return st;
  std::vector<int32_t> xs;
  host_columns(pl.job, pl.kq, &xs);
  if (x_of_col) {
    const uint64_t n = std::min<uint64_t>(cap, xs.size());
    memcpy(x_of_col, xs.data(), n * sizeof(int32_t));
  }
  return CS_OK;
}

extern "C" cs_status cs_rows(const cs_job* job, uint64_t* m_of_row, uint64_t cap) {
  Plan pl;
  cs_status st = make_plan(job, nullptr, 256, &pl);
  if (st) return st;
  uint64_t r = 0;
  for (uint64_t o = 0; o < pl.job.m_inc && r < cap; ++o) {
    const uint64_t m = pl.job.m_start + o;
    bool ok = true;
    for (uint32_t q : pl.dq)
      if (m % q == 0) { ok = false; break; }
    if (ok) {
      if (m_of_row) m_of_row[r] = m;
      ++r;
    }
  }
  return CS_OK;
}

namespace {

PrimeWs prime_ws_of(const Plan& pl, uint8_t* ws) {
  PrimeWs pw;
  const WsLayout& L = pl.ws;
  pw.base = reinterpret_cast<uint32_t*>(ws + L.base);
  pw.n_base = reinterpret_cast<uint32_t*>(ws + L.n_base);
  pw.flags = reinterpret_cast<uint32_t*>(ws + L.flags);
  pw.seg_count = reinterpret_cast<uint32_t*>(ws + L.seg_count);
  pw.seg_off = reinterpret_cast<uint64_t*>(ws + L.seg_off);
  pw.primes = reinterpret_cast<uint64_t*>(ws + L.primes);
  pw.n_primes = reinterpret_cast<uint64_t*>(ws + L.n_primes);
  pw.cap = pl.cap;
  if (pl.isq) {
    pw.base2 = reinterpret_cast<uint64_t*>(ws + L.base2);
    pw.n_base2 = reinterpret_cast<uint64_t*>(ws + L.n_base2);
    pw.flags2 = reinterpret_cast<uint32_t*>(ws + L.flags2);
    pw.seg_count2 = reinterpret_cast<uint32_t*>(ws + L.seg_count2);
    pw.seg_off2 = reinterpret_cast<uint64_t*>(ws + L.seg_off2);
    pw.cap2 = pl.cap2;
    pw.isq = pl.isq;
  }
  return pw;
}

struct AuxStream;
cs_status aux_clear(const Plan& pl, JobDev* jdp, uint32_t* bitmap, uint32_t* counts, hipStream_t s, int n_cu,
                    AuxStream* aux);
cs_status aux_join(AuxStream* aux, hipStream_t s);

// aux (optional): a second stream that clears the outputs and the byte counters beside the prime
// sieve (pure stores against the sieve's LDS work); `s` waits for it before returning.
cs_status prepare_planned(const Plan& pl, uint8_t* ws, hipStream_t s, int n_cu, AuxStream* aux = nullptr,
                          uint32_t* bitmap = nullptr, uint32_t* counts = nullptr) {
  const WsLayout& L = pl.ws;
  JobCtrl* ctrl = reinterpret_cast<JobCtrl*>(ws + L.ctrl);
  JobDev* jdp = reinterpret_cast<JobDev*>(ws + L.jobdev);
  PrimeWs pw = prime_ws_of(pl, ws);
  JobDev jd = make_jobdev(pl, ws, pw.primes, pw.n_primes);
  CS_TRY(launch_zero_ctrl(ctrl, s));
  CS_TRY(launch_write_job(jd, jdp, s));
  if (aux) CS_TRY(aux_clear(pl, jdp, bitmap, counts, s, n_cu, aux));
  CS_TRY(launch_primes(pl.Lp, pw, s));
  CS_TRY(launch_prep_tables(jdp, 1, s));
  CS_TRY(launch_kmod(jdp, 1, reinterpret_cast<uint64_t*>(ws + L.lim_base), pi_upper(pl.job.limit), n_cu, s));
  CS_TRY(launch_rows_cols(jdp, 1, pl.job.m_inc, pl.job.sl, n_cu, s));
  if (!pl.dpre.empty()) {
    CS_TRY(launch_upload(ws + L.dpre, pl.dpre.data(), pl.dpre.size() * 2ull, s));
    CS_TRY(launch_upload(ws + L.dres, pl.dres.data(), pl.dres.size() * 2ull, s));
  }
  if (pl.dpat_on) CS_TRY(launch_dpattern(jdp, 1, pl.phi_d, pl.row_words, s));
  if (aux) return aux_join(aux, s);
  if (pl.scatter_bytes) CS_TRY(launch_zero_bytes(jdp, 1, pl.n_m * (uint64_t)pl.row_words, n_cu, s));
  return CS_OK;
}

// HIP events around the last k_large launch of each workspace (read by cs_diag_read).  One pair
// per workspace address, created on first use and kept for the life of the process.
struct LargeEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  bool recorded = false;
};
std::mutex g_ev_mu;
std::map<const void*, LargeEvents> g_large_ev;

LargeEvents* large_events(const void* ws) {
  std::lock_guard<std::mutex> lk(g_ev_mu);
  LargeEvents& e = g_large_ev[ws];
  if (!e.start && (hipEventCreate(&e.start) != hipSuccess || hipEventCreate(&e.stop) != hipSuccess)) return nullptr;
  return &e;
}

// A second stream per device for running the small branch beside the large one (default
// priority, non-blocking), created on first use and kept for the life of the process, with a
// fork/join event pair per calling thread.
struct AuxStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_aux_mu;
std::map<std::pair<int, std::thread::id>, AuxStream> g_aux;

AuxStream* aux_stream() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_aux_mu);
  AuxStream& a = g_aux[{dev, std::this_thread::get_id()}];
  if (!a.s) {
    if (hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking) != hipSuccess) { a.s = nullptr; return nullptr; }
    if (hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&a.join, hipEventDisableTiming) != hipSuccess)
      return nullptr;
  }
  return &a;
}

// The clears of prepare_planned on the second stream: the outputs (when given) and the byte
// counters, after the job descriptor is written on `s`.
cs_status aux_clear(const Plan& pl, JobDev* jdp, uint32_t* bitmap, uint32_t* counts, hipStream_t s, int n_cu,
                    AuxStream* aux) {
  CS_TRY(hipEventRecord(aux->fork, s));
  CS_TRY(hipStreamWaitEvent(aux->s, aux->fork, 0));
  if (bitmap && pl.n_m > 0) {
    CS_TRY(launch_fill_u32(bitmap, pl.n_m * (uint64_t)pl.row_words, 0u, aux->s));
    CS_TRY(launch_fill_u32(counts, pl.n_m, 0u, aux->s));
  }
  if (pl.scatter_bytes) CS_TRY(launch_zero_bytes(jdp, 1, pl.n_m * (uint64_t)pl.row_words, n_cu, aux->s));
  CS_TRY(hipEventRecord(aux->join, aux->s));
  return CS_OK;
}

cs_status aux_join(AuxStream* aux, hipStream_t s) {
  CS_TRY(hipStreamWaitEvent(s, aux->join, 0));
  return CS_OK;
}

// own_stream_only: everything on `s`, with no second stream and no timing events (the entry point
// that allocates nothing creates neither).
// wide: the range lies at or above the plan's wide_lo; its large primes take the 64-bit path.
// fold_keep: no later call adds to the byte counters before the next preparation clears them, so
// the fold need not clear them back.
cs_status range_core(const Plan& pl, uint64_t p_lo, uint64_t p_hi, uint32_t* bitmap, uint32_t* counts,
                     uint8_t* ws, hipStream_t s, uint32_t branches, bool own_stream_only, bool wide,
                     bool fold_keep = false) {
  const WsLayout& L = pl.ws;
  JobDev* jdp = reinterpret_cast<JobDev*>(ws + L.jobdev);
  PrimeWs pw = prime_ws_of(pl, ws);
  JobDev jd = make_jobdev(pl, ws, pw.primes, pw.n_primes);
  jd.p_lo = p_lo;
  jd.p_hi = p_hi;
  jd.bitmap = bitmap;
  jd.counts = counts;
  jd.branches = branches;
  jd.fold_keep = fold_keep ? 1u : 0u;
  fill_tiers(pl, p_lo, p_hi, &jd);
  // With the byte counters or the list the large branch writes only its counters or cells until
  // the fold or the grouping, so the small branch can run beside it on a second stream.  With the
  // list, hits beyond a full pool are OR-ed into the bitmap by the large branch itself, so the small
  // branch then merges its tiles with atomics.
  hipStreamCaptureStatus cap0 = hipStreamCaptureStatusNone;
  AuxStream* aux = nullptr;
  if (!own_stream_only && branches == CS_BRANCH_ALL && (pl.scatter_bytes || pl.scatter_list) && pl.n_m > 0 &&
      hipStreamIsCapturing(s, &cap0) == hipSuccess && cap0 == hipStreamCaptureStatusNone)
    aux = aux_stream();
  if (aux && pl.scatter_list) jd.small_atomic = 1;
  uint64_t* items_base = reinterpret_cast<uint64_t*>(ws + L.items_base);
  CS_TRY(launch_write_job(jd, jdp, s));
  CS_TRY(launch_prep_bounds(jdp, 1, s));
  CS_TRY(launch_items_scan(jdp, 1, items_base, s));
  if (pl.n_m == 0) return CS_OK;
  const uint64_t units = (uint64_t)pl.n_windows * pl.n_slices;
  if (aux) {
    CS_TRY(hipEventRecord(aux->fork, s));
    CS_TRY(hipStreamWaitEvent(aux->s, aux->fork, 0));
  }
  hipStream_t s_small = aux ? aux->s : s;
  if (branches != CS_BRANCH_LARGE && !aux)
    CS_TRY(launch_small(jdp, 1, units, pl.lds_bytes, pl.lds_ct_words, pl.small_blocks, s_small, pl.small_hit_rows));
  JobCtrl* ctrl = reinterpret_cast<JobCtrl*>(ws + L.ctrl);
  if (branches != CS_BRANCH_SMALL) {
    if (pl.scatter_list) {
      CS_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.list_cursor), 2, 0u, s));
      CS_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.bkt_count), pl.n_bkt + 1ull, 0u, s));
      CS_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.list_super), kListSupers + 1ull, 0u, s));
    }
    const uint32_t kind = pl.scatter_list ? 2u : (pl.scatter_bytes ? 1u : 0u);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    LargeEvents* ev = nullptr;
    if (!own_stream_only && hipStreamIsCapturing(s, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone)
      ev = large_events(ws);
    if (ev) CS_TRY(hipEventRecord(ev->start, s));
    CS_TRY(launch_large(jdp, 1, items_base, ctrl->diag, &ctrl->dec[0][0], pl.large_blocks, pl.large_lds_bytes,
                        pl.large_lds_ct_words, (uint32_t)pl.dpre.size(), kind, pl.large_mode, s, wide));
    if (ev) {
      CS_TRY(hipEventRecord(ev->stop, s));
      ev->recorded = true;
    }
    if (aux) {   // small branch queued after the large kernel so the large one starts first
      CS_TRY(launch_small(jdp, 1, units, pl.lds_bytes, pl.lds_ct_words, pl.small_blocks, aux->s, pl.small_hit_rows));
      CS_TRY(hipEventRecord(aux->join, aux->s));
      CS_TRY(hipStreamWaitEvent(s, aux->join, 0));
    }
    if (pl.scatter_bytes) CS_TRY(launch_fold_bytes(jdp, 1, pl.n_m, device_cu_count(), s));
    if (pl.scatter_list) CS_TRY(launch_list_group(jdp, pl.list_chunks, pl.n_bkt, pl.bkt_rows, pl.super_shift, pl.row_words, s));
  }
  return CS_OK;
}

// The primes of [p_lo, p_hi]: below wide_lo with the fp64 arithmetic, from wide_lo on (large
// primes only, since the threshold stays below it) with the 64-bit arithmetic.
cs_status range_planned(const Plan& pl, uint64_t p_lo, uint64_t p_hi, uint32_t* bitmap, uint32_t* counts,
                        uint8_t* ws, hipStream_t s, uint32_t branches, bool own_stream_only = false,
                        bool fold_keep = false) {
  const uint64_t wl = pl.wide_lo;
  if (p_hi < wl || pl.job.limit < wl)
    return range_core(pl, p_lo, p_hi, bitmap, counts, ws, s, branches, own_stream_only, false, fold_keep);
  if (p_lo < wl) {
    cs_status st = range_core(pl, p_lo, wl - 1, bitmap, counts, ws, s, branches, own_stream_only, false);
    if (st) return st;
  }
  if (branches == CS_BRANCH_SMALL) return CS_OK;
  return range_core(pl, std::max(p_lo, wl), p_hi, bitmap, counts, ws, s, CS_BRANCH_LARGE, own_stream_only, true);
}

}  // namespace

extern "C" cs_status cs_prepare(const cs_job* job, const cs_tune* tune, void* d_ws, uint64_t ws_bytes,
                                void* stream) {
  Plan pl;
  const int n_cu = device_cu_count();
  cs_status st = make_plan(job, tune, n_cu, &pl);
  if (st) return st;
  if (!d_ws) return CS_EINVAL;
  if (ws_bytes < pl.ws.total) return CS_ERANGE;
  return prepare_planned(pl, static_cast<uint8_t*>(d_ws), (hipStream_t)stream, n_cu);
}

extern "C" cs_status cs_sieve_range(const cs_job* job, const cs_tune* tune, uint64_t p_lo, uint64_t p_hi,
                                    uint32_t* d_bitmap, uint32_t* d_counts, void* d_ws, uint64_t ws_bytes,
                                    void* stream) {
  Plan pl;
  const int n_cu = device_cu_count();
  cs_status st = make_plan(job, tune, n_cu, &pl);
  if (st) return st;
  if (!d_ws || (pl.n_m > 0 && (!d_bitmap || !d_counts))) return CS_EINVAL;
  if (ws_bytes < pl.ws.total) return CS_ERANGE;
  const uint32_t branches = tune ? tune->branches : CS_BRANCH_ALL;
  if (branches > CS_BRANCH_LARGE) return CS_EINVAL;
  if (p_hi < p_lo) return CS_OK;
  return range_planned(pl, p_lo, p_hi, d_bitmap, d_counts, static_cast<uint8_t*>(d_ws), (hipStream_t)stream,
                       branches);
}

extern "C" cs_status cs_sieve(const cs_job* job, const cs_tune* tune, uint32_t* d_bitmap, uint32_t* d_counts,
                              void* d_ws, uint64_t ws_bytes, void* stream) {
  Plan pl;
  const int n_cu = device_cu_count();
  cs_status st = make_plan(job, tune, n_cu, &pl);
  if (st) return st;
  if (!d_ws || (pl.n_m > 0 && (!d_bitmap || !d_counts))) return CS_EINVAL;
  if (ws_bytes < pl.ws.total) return CS_ERANGE;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  // the outputs and the byte counters are cleared on a second stream beside the prime sieve
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  AuxStream* aux = nullptr;
  if (pl.n_m > 0 && hipStreamIsCapturing(s, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone)
    aux = aux_stream();
  if (pl.n_m > 0 && !aux) {
    CS_TRY(launch_fill_u32(d_bitmap, pl.n_m * (uint64_t)pl.row_words, 0u, s));
    CS_TRY(launch_fill_u32(d_counts, pl.n_m, 0u, s));
  }
  st = prepare_planned(pl, ws, s, n_cu, aux, d_bitmap, d_counts);
  if (st) return st;
  // one range call over the whole prime range: its fold is the counters' last use in this call
  // (the wide part, when there is one, adds to them after the first part's fold)
  const bool keep = pl.job.limit < pl.wide_lo;
  return range_planned(pl, 2, pl.job.limit, d_bitmap, d_counts, ws, s, CS_BRANCH_ALL, false, keep);
}

namespace {
cs_status chunked_planned(const Plan& pl, uint64_t p_lo, uint64_t p_hi, uint32_t* d_bitmap, uint32_t* d_counts,
                          uint8_t* ws, hipStream_t s, int n_cu) {
  // the first chunk [0, span) (every prime <= P, so K's groups and the row and column tables
  // come from it) is an ordinary preparation with a prime table of one chunk
  cs_status st = prepare_planned(pl, ws, s, n_cu);
  if (st) return st;
  const uint64_t limit = pl.job.limit;
  const uint64_t lo = std::max<uint64_t>(p_lo, 2), hi_all = std::min(p_hi, limit);
  const uint64_t step = pl.span ? pl.span : limit + 1;
  // from the chunk that holds p_lo (chunks below it hold no prime of the range)
  for (uint64_t a = lo / step * step; a <= hi_all; a += step) {
    const uint64_t hi = std::min<uint64_t>(a + step - 1, limit);
    if (a > 0) {
      PrimeWs pw = prime_ws_of(pl, ws);
      JobDev* jdp = reinterpret_cast<JobDev*>(ws + pl.ws.jobdev);
      CS_TRY(launch_primes_range(a >> kSegLog, hi, pw, s));
      CS_TRY(launch_chunk_bounds(jdp, s));
      CS_TRY(launch_kmod(jdp, 1, reinterpret_cast<uint64_t*>(ws + pl.ws.lim_base), pl.cap, n_cu, s));
    }
    st = range_planned(pl, std::max<uint64_t>(a, lo), std::min(hi, hi_all), d_bitmap, d_counts, ws, s,
                       CS_BRANCH_ALL);
    if (st) return st;
    if (a + step < a) break;                        // (no wrap-around for limits near 2^64)
  }
  return CS_OK;
}
}  // namespace

extern "C" cs_status cs_sieve_chunked_range(const cs_job* job, const cs_tune* tune, uint64_t span, uint64_t p_lo,
                                            uint64_t p_hi, uint32_t* d_bitmap, uint32_t* d_counts, void* d_ws,
                                            uint64_t ws_bytes, void* stream) {
  if (!span) return CS_EINVAL;
  Plan pl;
  const int n_cu = device_cu_count();
  cs_status st = make_plan(job, tune, n_cu, &pl, true, true, true, span);
  if (st) return st;
  if (!d_ws || (pl.n_m > 0 && (!d_bitmap || !d_counts))) return CS_EINVAL;
  if (ws_bytes < pl.ws.total) return CS_ERANGE;
  if (p_hi < p_lo) return CS_OK;
  return chunked_planned(pl, p_lo, p_hi, d_bitmap, d_counts, static_cast<uint8_t*>(d_ws), (hipStream_t)stream, n_cu);
}

extern "C" cs_status cs_sieve_chunked(const cs_job* job, const cs_tune* tune, uint64_t span, uint32_t* d_bitmap,
                                      uint32_t* d_counts, void* d_ws, uint64_t ws_bytes, void* stream) {
  if (!span) return CS_EINVAL;
  Plan pl;
  const int n_cu = device_cu_count();
  cs_status st = make_plan(job, tune, n_cu, &pl, true, true, true, span);
  if (st) return st;
  if (!d_ws || (pl.n_m > 0 && (!d_bitmap || !d_counts))) return CS_EINVAL;
  if (ws_bytes < pl.ws.total) return CS_ERANGE;
  hipStream_t s = (hipStream_t)stream;
  if (pl.n_m > 0) {
    CS_TRY(launch_fill_u32(d_bitmap, pl.n_m * (uint64_t)pl.row_words, 0u, s));
    CS_TRY(launch_fill_u32(d_counts, pl.n_m, 0u, s));
  }
  return chunked_planned(pl, 2, pl.job.limit, d_bitmap, d_counts, static_cast<uint8_t*>(d_ws), s, n_cu);
}

extern "C" cs_status cs_diag_read(const void* d_ws, cs_diag* out, void* stream) {
  if (!d_ws || !out) return CS_EINVAL;
  // every workspace layout puts the control block first (WsLayout::ctrl == 0)
  hipStream_t s = (hipStream_t)stream;
  if (hipStreamSynchronize(s) != hipSuccess) return CS_EDEVICE;
  JobCtrl c;
  if (hipMemcpy(&c, d_ws, sizeof(JobCtrl), hipMemcpyDeviceToHost) != hipSuccess) return CS_EDEVICE;
  out->n_primes = c.diag[D_NPRIMES];
  out->small_primes = c.diag[D_SMALL_PRIMES];
  out->large_primes = c.diag[D_LARGE_PRIMES];
  out->small_pairs = c.diag[D_SMALL_PAIRS];
  out->small_marks = c.diag[D_SMALL_MARKS];
  out->large_raw_hits = c.diag[D_LARGE_RAW];
  out->large_hits = c.diag[D_LARGE_HITS];
  out->g_calls = c.diag[D_G_CALLS];
  out->g_levels = c.diag[D_G_LEVELS];
  out->error_flags = c.diag[D_ERROR] | c.error;
  for (int i = 0; i < kDecades; ++i) {
    out->dec_primes[i] = c.dec[DC_PRIMES][i];
    out->dec_raw_hits[i] = c.dec[DC_RAW][i];
    out->dec_hits[i] = c.dec[DC_HITS][i];
    out->dec_solves[i] = c.dec[DC_SOLVES][i];
    out->dec_levels[i] = c.dec[DC_LEVELS][i];
  }
  out->large_kernel_ms = 0.0;
  {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    auto it = g_large_ev.find(d_ws);
    float ms = 0.f;
    if (it != g_large_ev.end() && it->second.recorded &&
        hipEventElapsedTime(&ms, it->second.start, it->second.stop) == hipSuccess)
      out->large_kernel_ms = ms;
  }
  return out->error_flags ? CS_EDEVICE : CS_OK;
}

// ---------------------------------------------------------------------------------------------
// Stand-alone prime table and K mod p.
// ---------------------------------------------------------------------------------------------
namespace {
struct PrimeOnlyLayout {
  uint64_t n_base, base, flags, seg_count, seg_off, total, n_seg, cap;
};
PrimeOnlyLayout prime_only_layout(uint64_t limit) {
  PrimeOnlyLayout L;
  uint64_t o = 0;
  auto take = [&](uint64_t b) { uint64_t at = o; o = (o + std::max<uint64_t>(b, 8) + 255) & ~255ull; return at; };
  L.n_seg = (limit >> kSegLog) + 1;
  L.cap = pi_upper(limit);
  L.n_base = take(8);
  L.base = take(kBaseCap * 4ull);
  L.flags = take(L.n_seg * kSegWords * 4ull);
  L.seg_count = take(L.n_seg * 4ull);
  L.seg_off = take(L.n_seg * 8ull);
  L.total = o;
  return L;
}
}  // namespace

extern "C" cs_status cs_primes_ws(uint64_t limit, uint64_t* cap_out, uint64_t* ws_bytes_out) {
  if (limit < 2) return CS_EINVAL;
  if (limit >= kWideLo) return CS_ERANGE;
  PrimeOnlyLayout L = prime_only_layout(limit);
  if (cap_out) *cap_out = L.cap;
  if (ws_bytes_out) *ws_bytes_out = L.total;
  return CS_OK;
}

extern "C" cs_status cs_primes(uint64_t limit, uint64_t* d_primes, uint64_t cap, uint64_t* d_count, void* d_ws,
                               uint64_t ws_bytes, void* stream) {
  if (limit < 2 || !d_primes || !d_count || !d_ws) return CS_EINVAL;
  if (limit >= kWideLo) return CS_ERANGE;
  PrimeOnlyLayout L = prime_only_layout(limit);
  if (cap < L.cap || ws_bytes < L.total) return CS_ERANGE;
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  PrimeWs pw;
  pw.base = reinterpret_cast<uint32_t*>(ws + L.base);
  pw.n_base = reinterpret_cast<uint32_t*>(ws + L.n_base);
  pw.flags = reinterpret_cast<uint32_t*>(ws + L.flags);
  pw.seg_count = reinterpret_cast<uint32_t*>(ws + L.seg_count);
  pw.seg_off = reinterpret_cast<uint64_t*>(ws + L.seg_off);
  pw.primes = d_primes;
  pw.n_primes = d_count;
  pw.cap = cap;
  CS_TRY(launch_primes(limit, pw, (hipStream_t)stream));
  return CS_OK;
}

extern "C" cs_status cs_kmod(uint32_t P, uint64_t d, const uint64_t* d_primes, uint64_t n, uint64_t* d_out,
                             void* d_ws, uint64_t ws_bytes, void* stream) {
  cs_job j;
  memset(&j, 0, sizeof(j));
  j.P = P; j.d = d; j.m_start = 1; j.m_inc = 1; j.sl = 1; j.limit = 2;
  Plan pl;
  cs_status st = make_plan(&j, nullptr, 256, &pl);
  if (st == CS_EINVAL) {
    // sl < m_start*K may fail for K = 1 (d = P#); only P and d matter here
    j.m_start = 2;
    st = make_plan(&j, nullptr, 256, &pl);
  }
  if (st) return st;
  if ((n > 0 && (!d_primes || !d_out)) || !d_ws) return CS_EINVAL;
  std::vector<uint64_t> groups;
  uint64_t g = 1;
  for (uint32_t q : pl.kq) {
    if (g > (kGroupMax - 1) / q) { groups.push_back(g); g = q; }
    else g *= q;
  }
  if (g > 1) groups.push_back(g);
  if (ws_bytes < std::max<uint64_t>(groups.size(), 1) * 8ull) return CS_ERANGE;
  if (n == 0) return CS_OK;
  hipStream_t s = (hipStream_t)stream;
  if (!groups.empty()) CS_TRY(launch_upload(d_ws, groups.data(), groups.size() * 8ull, s));
  CS_TRY(launch_kmod_list(d_primes, n, static_cast<const uint64_t*>(d_ws), (uint32_t)groups.size(), d_out,
                          device_cu_count(), s));
  return CS_OK;
}

extern "C" cs_status cs_kmod_ws(uint32_t P, uint64_t d, uint64_t* ws_bytes_out) {
  cs_job j;
  memset(&j, 0, sizeof(j));
  j.P = P; j.d = d; j.m_start = 2; j.m_inc = 1; j.sl = 1; j.limit = 2;
  Plan pl;
  cs_status st = make_plan(&j, nullptr, 256, &pl);
  if (st) return st;
  if (ws_bytes_out) *ws_bytes_out = (pl.kq.size() + 1) * 8ull;
  return CS_OK;
}

extern "C" cs_status cs_probe_scatter(uint32_t* d_buf, uint64_t words, uint64_t n_ops, uint32_t slices, uint32_t op,
                                      uint64_t seed, void* stream) {
  if (!d_buf || op > 2 || slices == 0 || slices > 16) return CS_EINVAL;
  if (words < slices || words / slices == 0) return CS_EINVAL;
  if (n_ops == 0) return CS_OK;
  CS_TRY(launch_probe_scatter(d_buf, words, n_ops, slices, op, seed, device_cu_count(), (hipStream_t)stream));
  return CS_OK;
}

// ---------------------------------------------------------------------------------------------
// The whole sieve with a workspace the library holds: for callers that cannot allocate device
// memory (code under graph capture, serving loops, harnesses that forbid hipMalloc).  The
// workspace is a static device array of kScratchBytes in this code object, one copy per device;
// host code uses only the device address of the current device's copy, taken once per device.
// ---------------------------------------------------------------------------------------------
static constexpr uint64_t kScratchBytes = 256ull << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, uint8_t*> g_scratch;   // device -> device address of its copy of `scratch`

cs_status scratch_ptr(uint8_t** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CS_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it != g_scratch.end()) {
    *out = it->second;
    return CS_OK;
  }
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return CS_EDEVICE;
  g_scratch[dev] = static_cast<uint8_t*>(p);
  *out = static_cast<uint8_t*>(p);
  return CS_OK;
}
}  // namespace

extern "C" uint64_t cs_scratch_bytes(void) { return kScratchBytes; }

extern "C" cs_status cs_sieve_noalloc(const cs_job* job, const cs_tune* tune, uint32_t* d_bitmap, uint32_t* d_counts,
                                      void* stream) {
  Plan pl;
  const int n_cu = device_cu_count();
  cs_status st = make_plan(job, tune, n_cu, &pl);
  if (st) return st;
  if (pl.n_m > 0 && (!d_bitmap || !d_counts)) return CS_EINVAL;
  if (pl.ws.total > kScratchBytes) return CS_ERANGE;
  uint8_t* ws = nullptr;
  st = scratch_ptr(&ws);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if (pl.n_m > 0) {
    CS_TRY(launch_fill_u32(d_bitmap, pl.n_m * (uint64_t)pl.row_words, 0u, s));
    CS_TRY(launch_fill_u32(d_counts, pl.n_m, 0u, s));
  }
  st = prepare_planned(pl, ws, s, n_cu);
  if (st) return st;
  return range_planned(pl, 2, pl.job.limit, d_bitmap, d_counts, ws, s, CS_BRANCH_ALL, true);
}

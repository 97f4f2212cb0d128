// Serving: a request loop that admits sieve jobs by device memory, keeps the prime table and
// per-(P, d) K mod p tables resident, and runs continuous batching.
//
// Each job is split into prime-range chunks: the large primes in C ranges of about equal prime
// count, the first of which also takes the small primes (p <= thr), whose branch runs on a second
// stream beside the large one.  One iteration
// of the server is one fused launch sequence that advances every active job by one chunk
// (OR-ing and adding into its outputs; Section 3's marks are order independent).  Jobs that
// arrive while others run are admitted at the next iteration when a slot and memory are free,
// so their work shares the same kernels as the jobs already in flight.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/csieve.h"
#include "batch_internal.h"
#include "device.h"
#include "launch.h"
#include "plan.h"

using namespace cs;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

uint64_t a256(uint64_t x) { return (x + 255) & ~255ull; }

// First-fit allocator over one device allocation (offsets, 256-byte granules).
class Arena {
 public:
  void init(uint64_t cap) {
    free_.clear();
    if (cap) free_[0] = cap;
    used_ = 0;
  }
  bool alloc(uint64_t size, uint64_t* off) {
    size = a256(std::max<uint64_t>(size, 256));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < size) continue;
      *off = it->first;
      const uint64_t rest = it->second - size;
      const uint64_t at = it->first + size;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += size;
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t size) {
    size = a256(std::max<uint64_t>(size, 256));
    used_ -= size;
    auto it = free_.emplace(off, size).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t used() const { return used_; }

 private:
  std::map<uint64_t, uint64_t> free_;
  uint64_t used_ = 0;
};

struct KEntry {
  uint32_t P;
  uint64_t d, limit, off, bytes;
  int refs;
  bool ready;
  double last_use;
};
// Cache entries live in a map keyed by a stable id (jobs hold ids, never positions).

enum JobState { S_QUEUED = 0, S_ACTIVE = 1, S_DONE = 2, S_ERROR = -1 };

struct SJob {
  cs_job job;
  Plan plan;
  int state = S_QUEUED;
  bool prepped = false;
  double t_submit = 0, t_admit = 0, t_done = 0;
  uint64_t off_tab = 0, bytes_tab = 0, off_out = 0, bytes_out = 0;
  uint64_t kentry = 0;              // id of the K mod p table (0: none)
  uint32_t chunk = 0;
  uint32_t lane = 0;                // 0: the short lane, 1: the long lane
  std::vector<uint64_t> bounds;   // chunk c covers primes in (bounds[c], bounds[c+1]]
  JobDev jd;
};

// One lane of the server: its own loop thread, streams, descriptor arrays, queue and active set.
// With two lanes the jobs estimated to take long run in the second one, so that the iterations of
// the others (which complete a job per iteration) do not wait for them.
struct Lane {
  hipStream_t stream = nullptr;
  hipStream_t aux = nullptr;           // the small branch beside the large one (default priority)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  JobDev* run_dev = nullptr;
  JobDev* prep_dev = nullptr;
  uint64_t* lim_base = nullptr;
  uint64_t* items_base = nullptr;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> active;
  std::thread th;
};

// Prime value below which about `frac` of the primes up to `hi` (and above lo) lie.
uint64_t prime_quantile(uint64_t lo, uint64_t hi, double frac) {
  auto pc = [](double x) { return x < 3 ? 0.0 : x / log(x); };
  const double target = pc((double)lo) + frac * (pc((double)hi) - pc((double)lo));
  double a = (double)lo, b = (double)hi;
  for (int it = 0; it < 80; ++it) {
    const double m = 0.5 * (a + b);
    if (pc(m) < target) a = m; else b = m;
  }
  return (uint64_t)b;
}

}  // namespace

struct cs_server {
  cs_server_config cfg;
  int device = 0;
  int n_cu = 256;
  Lane lane[2];
  uint32_t n_lanes = 1;
  uint8_t* arena_mem = nullptr;
  uint8_t* fixed_mem = nullptr;
  Arena arena;
  PrimeWs pw{};
  unsigned long long* diag = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  bool failed = false;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, SJob> jobs;
  std::map<uint64_t, KEntry> kcache;
  uint64_t next_kid = 1;
  cs_server_counters st{};
};

namespace {

uint64_t job_bytes(const Plan& pl) {
  return a256(pl.ws.total) + a256(pl.n_m * (uint64_t)pl.row_words * 4ull) + a256(pl.n_m * 4ull);
}

uint64_t kmod_bytes(uint64_t limit) { return a256(pi_upper(limit) * 8ull); }

// Small/large threshold of a served three-gap job, per column of the interval.  A prime p in the
// small branch costs about n_m residue steps of c_pair = 1.25 ps; in the large branch it costs
// about n_m n_x / p hit atomics of c_hit = 55 ps (plus a setup that is small beside n_m c_pair).
// A lone job hides its small branch beside the large one, but the server's iterations run many
// jobs' small and large branches at once, where the two add up: their sum is least at
// p = n_x c_hit / c_pair, about 44 n_x (measured on the mixed jobs alone: 15% less device time
// than the lone job's 30 S).
constexpr uint64_t kServerThrPerColumn = 44;

// A job whose large branch forms K mod p itself keeps a table for its small primes in its own
// tables; any other job shares one K mod p table per (P, d) across jobs.  The job's tables hold
// byte counters for its large hits (one atomic per hit instead of two) where they are exact and
// the job then takes at most a quarter of the budget; the scatter ATOMIC keeps them out.
cs_status plan_for_server(const cs_server* s, const cs_job* job, Plan* pl) {
  cs_tune t = s->cfg.tune;
  if (t.scatter != CS_SCATTER_ATOMIC) t.scatter = CS_SCATTER_AUTO;
  if (t.thr == 0 && t.large_mode == CS_LARGE_THREE_GAP) {
    const cs_status st = make_plan(job, &t, s->n_cu, pl, false, true, false);
    if (st) return st;
    t.thr = std::max<uint64_t>(1, kServerThrPerColumn * pl->n_x);
  }
  for (int bytes = t.scatter == CS_SCATTER_AUTO ? 1 : 0; bytes >= 0; --bytes) {
    cs_status st = make_plan(job, &t, s->n_cu, pl, false, true, bytes != 0);
    if (st) return st;
    if (!pl->kmod_fused) {
      st = make_plan(job, &t, s->n_cu, pl, false, false, bytes != 0);
      if (st) return st;
    }
    if (!pl->scatter_bytes ||
        job_bytes(*pl) + (pl->kmod_fused ? 0 : kmod_bytes(job->limit)) <= s->cfg.budget_bytes / 4)
      break;
  }
  if (pl->Lp > s->cfg.max_limit) return CS_ERANGE;
  return CS_OK;
}

// Frees unreferenced K mod p tables, least recently used first, until `need` bytes fit.
bool make_room(cs_server* s, uint64_t need) {
  uint64_t off;
  while (true) {
    if (s->arena.alloc(need, &off)) {
      s->arena.release(off, need);
      return true;
    }
    auto victim = s->kcache.end();
    for (auto it = s->kcache.begin(); it != s->kcache.end(); ++it)
      if (it->second.refs == 0 && (victim == s->kcache.end() || it->second.last_use < victim->second.last_use))
        victim = it;
    if (victim == s->kcache.end()) return false;
    s->arena.release(victim->second.off, victim->second.bytes);
    s->kcache.erase(victim);
    s->st.kmod_evictions++;
  }
}

void set_chunks(cs_server* s, SJob& J);

// Admits a job whose tables hold its own (small-prime) K mod p: memory and descriptor only.
bool admit_own(cs_server* s, SJob& J) {
  const Plan& pl = J.plan;
  const uint64_t need = job_bytes(pl);
  if (!make_room(s, need + 256)) return false;
  uint64_t off_t = 0, off_o = 0;
  const uint64_t bt = a256(pl.ws.total);
  const uint64_t bo = need - bt;
  if (!s->arena.alloc(bt, &off_t)) return false;
  if (!s->arena.alloc(bo, &off_o)) { s->arena.release(off_t, bt); return false; }
  J.kentry = 0;
  J.off_tab = off_t;
  J.bytes_tab = bt;
  J.off_out = off_o;
  J.bytes_out = bo;
  uint8_t* ws = s->arena_mem + off_t;
  J.jd = make_jobdev(pl, ws, s->pw.primes, s->pw.n_primes);
  J.jd.prime_cap = s->pw.cap;
  J.jd.kmod_cached = 0;
  J.jd.bitmap = reinterpret_cast<uint32_t*>(s->arena_mem + off_o);
  J.jd.counts = reinterpret_cast<uint32_t*>(s->arena_mem + off_o + a256(pl.n_m * (uint64_t)pl.row_words * 4ull));
  set_chunks(s, J);
  return true;
}

// Tries to admit the job (memory, K mod p table, descriptor).  Called with the mutex held.
bool admit(cs_server* s, uint64_t ticket) {
  SJob& J = s->jobs[ticket];
  const Plan& pl = J.plan;
  // K mod p table for (P, d): reuse one whose limit covers this job's (prime indices agree); a job
  // that forms K mod p itself needs none
  uint64_t kid = 0;
  if (pl.kmod_fused) return admit_own(s, J);
  for (auto& kv : s->kcache) {
    const KEntry& e = kv.second;
    if (e.P == J.job.P && e.d == J.job.d && e.limit >= J.job.limit) { kid = kv.first; break; }
  }
  const uint64_t need_k = kid == 0 ? kmod_bytes(J.job.limit) : 0;
  const uint64_t need = job_bytes(pl);
  if (!make_room(s, need + need_k + 256)) return false;
  uint64_t off_k = 0, off_t = 0, off_o = 0;
  const uint64_t bt = a256(pl.ws.total);
  const uint64_t bo = need - bt;
  if (!s->arena.alloc(bt, &off_t)) return false;
  if (!s->arena.alloc(bo, &off_o)) { s->arena.release(off_t, bt); return false; }
  if (kid == 0) {
    if (!s->arena.alloc(need_k, &off_k)) {
      s->arena.release(off_t, bt);
      s->arena.release(off_o, bo);
      return false;
    }
    kid = s->next_kid++;
    s->kcache[kid] = KEntry{J.job.P, J.job.d, J.job.limit, off_k, need_k, 0, false, now_s()};
    s->st.kmod_builds++;
  } else {
    s->st.kmod_hits++;
  }
  KEntry& E = s->kcache[kid];
  E.refs++;
  E.last_use = now_s();
  J.kentry = kid;
  J.off_tab = off_t;
  J.bytes_tab = bt;
  J.off_out = off_o;
  J.bytes_out = bo;
  uint8_t* ws = s->arena_mem + off_t;
  J.jd = make_jobdev(pl, ws, s->pw.primes, s->pw.n_primes);
  J.jd.prime_cap = s->pw.cap;
  J.jd.kmod = reinterpret_cast<uint64_t*>(s->arena_mem + E.off);
  J.jd.kmod_cached = E.ready ? 1u : 0u;
  J.jd.bitmap = reinterpret_cast<uint32_t*>(s->arena_mem + off_o);
  J.jd.counts = reinterpret_cast<uint32_t*>(s->arena_mem + off_o + a256(pl.n_m * (uint64_t)pl.row_words * 4ull));
  set_chunks(s, J);
  return true;
}

// The job's chunks (the large primes in ranges of about equal prime count, the small primes with
// the first), and the job marked active.
void set_chunks(cs_server* s, SJob& J) {
  const Plan& pl = J.plan;
  J.bounds.clear();
  J.bounds.push_back(1);
  const uint64_t thr = std::min<uint64_t>(pl.thr, J.job.limit);
  if (J.job.limit > thr) {
    const uint32_t C = std::max<uint32_t>(1, s->cfg.chunks);
    for (uint32_t c = 1; c < C; ++c) {
      const uint64_t v = prime_quantile(thr, J.job.limit, (double)c / C);
      if (v > J.bounds.back() && v > thr && v < J.job.limit) J.bounds.push_back(v);
    }
  }
  J.bounds.push_back(J.job.limit);
  J.chunk = 0;
  J.state = S_ACTIVE;
  J.prepped = false;
  J.t_admit = now_s();
  s->st.admitted++;
}

void retire(cs_server* s, SJob& J, int state) {
  s->arena.release(J.off_tab, J.bytes_tab);
  J.off_tab = J.bytes_tab = 0;
  auto it = s->kcache.find(J.kentry);
  if (it != s->kcache.end()) {
    it->second.refs--;
    if (J.prepped && state == S_DONE) it->second.ready = true;
    it->second.last_use = now_s();
  }
  J.kentry = 0;
  J.state = state;
  J.t_done = now_s();
  if (state == S_DONE) s->st.completed++;
  else s->st.failed++;
}

// One iteration: prepare the newly admitted jobs and advance every active job by one chunk.
bool iterate(cs_server* s, Lane& L, std::vector<SJob*>& act, bool* used_bytes) {
  hipStream_t st = L.stream;
  const uint32_t n = (uint32_t)act.size();
  std::vector<SJob*> fresh;
  for (SJob* J : act)
    if (!J->prepped) fresh.push_back(J);
  if (!fresh.empty()) {
    uint64_t kcap = 0, max_words = 0, max_m = 0;
    uint32_t max_sl = 0, max_phi = 0, max_rw = 0;
    for (uint32_t i = 0; i < fresh.size(); ++i) {
      SJob& J = *fresh[i];
      if (launch_write_job(J.jd, L.prep_dev + i, st) != hipSuccess) return false;
      if (!J.plan.dpre.empty() &&
          (launch_upload(s->arena_mem + J.off_tab + J.plan.ws.dpre, J.plan.dpre.data(), J.plan.dpre.size() * 2ull,
                         st) != hipSuccess ||
           launch_upload(s->arena_mem + J.off_tab + J.plan.ws.dres, J.plan.dres.data(), J.plan.dres.size() * 2ull,
                         st) != hipSuccess))
        return false;
      if (J.plan.dpat_on) {
        max_phi = std::max(max_phi, J.plan.phi_d);
        max_rw = std::max(max_rw, J.plan.row_words);
      }
      kcap += J.plan.kmod_fused ? std::min(pi_upper(J.job.limit), pi_upper(J.plan.thr)) : pi_upper(J.job.limit);
      max_words = std::max<uint64_t>(max_words, J.plan.n_m * (uint64_t)J.plan.row_words);
      max_m = std::max<uint64_t>(max_m, J.job.m_inc);
      max_sl = std::max(max_sl, J.job.sl);
    }
    const uint32_t nf = (uint32_t)fresh.size();
    if (launch_zero_ctrls(L.prep_dev, nf, st) != hipSuccess) return false;
    if (launch_fill_jobs(L.prep_dev, nf, max_words, st) != hipSuccess) return false;
    if (launch_prep_tables(L.prep_dev, nf, st) != hipSuccess) return false;
    if (launch_kmod(L.prep_dev, nf, L.lim_base, kcap, s->n_cu, st) != hipSuccess) return false;
    if (launch_rows_cols(L.prep_dev, nf, max_m, max_sl, s->n_cu, st) != hipSuccess) return false;
    if (launch_dpattern(L.prep_dev, nf, max_phi, max_rw, st) != hipSuccess) return false;
    // the byte counters start cleared; every fold clears them again
    if (launch_zero_bytes(L.prep_dev, nf, max_words, s->n_cu, st) != hipSuccess) return false;
    for (SJob* J : fresh) J->prepped = true;
  }
  // the byte counters when every job has them (a job without rows has no large items)
  bool bytes = true;
  uint64_t max_rows = 0;
  for (SJob* J : act) {
    if (J->plan.n_m && !J->plan.scatter_bytes) bytes = false;
    max_rows = std::max<uint64_t>(max_rows, J->plan.n_m);
  }
  // the sieve: every active job's current chunk, fused
  uint64_t units = 0;
  uint32_t lds = 0, max_ct = 0;
  for (SJob* J : act) max_ct = std::max(max_ct, J->plan.ct_words);
  const uint32_t lds_ct = max_ct * 8u <= kLdsCtMax ? max_ct : 0u;
  for (uint32_t i = 0; i < n; ++i) {
    SJob& J = *act[i];
    retile_small(J.plan, lds_ct, s->n_cu, &s->cfg.tune);
    JobDev jd = J.jd;
    jd.tile_rows = J.plan.tile_rows;
    jd.n_windows = J.plan.n_windows;
    jd.n_slices = J.plan.n_slices;
    jd.kmod_cached = 1;
    jd.p_lo = J.bounds[J.chunk] + 1;
    jd.p_hi = J.bounds[J.chunk + 1];
    fill_tiers(J.plan, jd.p_lo, jd.p_hi, &jd);
    jd.small_unit_base = units;
    jd.small_atomic = bytes ? 0u : 1u;   // with the counters the large branch leaves the bitmap alone
    if (J.chunk == 0) {
      units += (uint64_t)J.plan.n_windows * J.plan.n_slices;
      lds = std::max(lds, J.plan.lds_bytes);
    }
    if (launch_write_job(jd, L.run_dev + i, st) != hipSuccess) return false;
  }
  if (launch_prep_bounds(L.run_dev, n, st) != hipSuccess) return false;
  if (launch_items_scan(L.run_dev, n, L.items_base, st) != hipSuccess) return false;
  // the small branch on the second stream beside the large one: either the large branch writes
  // only its byte counters, folded in after both, or both merge into the bitmap and counts with
  // atomics (small_atomic); the order of their updates does not matter
  if (units) {
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(units, 1ull << 31);   // one workgroup per unit
    if (hipEventRecord(L.ev_fork, st) != hipSuccess || hipStreamWaitEvent(L.aux, L.ev_fork, 0) != hipSuccess)
      return false;
    if (launch_small(L.run_dev, n, units, lds, lds_ct, blocks, L.aux) != hipSuccess) return false;
  }
  if (launch_large(L.run_dev, n, L.items_base, s->diag, nullptr, (uint32_t)s->n_cu * kLargeBlocksPerCu, 0, 0, 0,
                   bytes ? 1u : 0u, s->cfg.tune.large_mode, st) != hipSuccess)
    return false;
  if (units && (hipEventRecord(L.ev_join, L.aux) != hipSuccess || hipStreamWaitEvent(st, L.ev_join, 0) != hipSuccess))
    return false;
  if (bytes && launch_fold_bytes(L.run_dev, n, max_rows, s->n_cu, st) != hipSuccess) return false;
  if (hipStreamSynchronize(st) != hipSuccess) return false;
  *used_bytes = bytes;
  return true;
}

void server_loop(cs_server* s, uint32_t li) {
  (void)hipSetDevice(s->device);
  Lane& L = s->lane[li];
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    // admission: queue order, as slots and memory allow
    while (!L.pending.empty() && L.active.size() < s->cfg.max_active) {
      const uint64_t t = L.pending.front();
      if (!admit(s, t)) break;
      L.pending.pop_front();
      L.active.push_back(t);
    }
    if (L.active.empty()) {
      s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
      continue;
    }
    std::vector<SJob*> act;
    for (uint64_t t : L.active) act.push_back(&s->jobs[t]);
    lk.unlock();
    bool used_bytes = false;
    const bool ok = iterate(s, L, act, &used_bytes);
    lk.lock();
    s->st.iterations++;
    if (used_bytes) s->st.bytes_iterations++;
    std::vector<uint64_t> keep;
    for (uint64_t t : L.active) {
      SJob& J = s->jobs[t];
      if (!ok) { retire(s, J, S_ERROR); continue; }
      J.chunk++;
      if (J.chunk + 1 >= J.bounds.size()) retire(s, J, S_DONE);
      else keep.push_back(t);
    }
    L.active.swap(keep);
    if (!ok) s->failed = true;
    s->cv_done.notify_all();
    s->cv_work.notify_all();          // memory freed here may admit the other lane's jobs
  }
}

// Estimated device time of a job alone (ms), from its plan: the large branch's hit atomics
// (n_m n_x (log log limit - log log thr) by Mertens' theorem, at about 1.8e10 per second) or its
// per-prime setup (about 45 ps per large prime), whichever is larger, plus part of the small
// branch (about 1.25 ps per (row, small prime) pair, largely hidden beside the large one).
double est_ms(const Plan& pl) {
  const cs_job& j = pl.job;
  if (pl.n_m == 0) return 0.0;
  const double thr = std::max<double>((double)std::min<uint64_t>(pl.thr, j.limit), 3.0);
  const double lim = std::max<double>((double)j.limit, thr);
  auto pc = [](double x) { return x < 3 ? 0.0 : x / log(x); };
  const double hits = (double)pl.n_m * pl.n_x * std::max(0.0, log(log(lim)) - log(log(thr)));
  const double large = std::max(hits / 1.8e10, (pc(lim) - pc(thr)) * 4.5e-11);
  const double small = (double)pl.n_m * pc(thr) * 1.25e-12;
  return 1e3 * (large + 0.3 * small);
}

void fill_info(const cs_server* s, const SJob& J, cs_ticket_info* out) {
  (void)s;
  memset(out, 0, sizeof(*out));
  out->state = J.state;
  const double t_end = J.t_done > 0 ? J.t_done : now_s();
  out->queued_s = (J.t_admit > 0 ? J.t_admit : t_end) - J.t_submit;
  out->latency_s = t_end - J.t_submit;
  out->n_m = J.plan.n_m;
  out->n_x = J.plan.n_x;
  out->row_words = J.plan.row_words;
}

}  // namespace

extern "C" cs_status cs_server_create(const cs_server_config* cfg, cs_server** out) {
  if (!cfg || !out || cfg->budget_bytes == 0 || cfg->max_active == 0 || cfg->max_limit < 2) return CS_EINVAL;
  if (!(cfg->long_ms >= 0.0)) return CS_EINVAL;
  if (cfg->max_limit >= kWideLo) return CS_ERANGE;
  *out = nullptr;
  cs_server* s = new (std::nothrow) cs_server();
  if (!s) return CS_ENOMEM;
  s->cfg = *cfg;
  if (hipGetDevice(&s->device) != hipSuccess) { delete s; return CS_EDEVICE; }
  s->n_cu = device_cu_count();
  s->n_lanes = cfg->long_ms > 0.0 ? 2u : 1u;
  // fixed memory: prime table up to max_limit, descriptors and prefix arrays per lane, counters
  const uint64_t n_seg = (cfg->max_limit >> kSegLog) + 1, cap = pi_upper(cfg->max_limit);
  const uint32_t na = cfg->max_active;
  uint64_t o = 0;
  auto take = [&](uint64_t b) { uint64_t at = o; o = a256(o + std::max<uint64_t>(b, 8)); return at; };
  const uint64_t o_nb = take(8), o_np = take(8), o_base = take(kBaseCap * 4ull), o_fl = take(n_seg * kSegWords * 4ull);
  const uint64_t o_sc = take(n_seg * 4ull), o_so = take(n_seg * 8ull), o_pr = take(cap * 8ull);
  uint64_t o_run[2], o_prep[2], o_lim[2], o_it[2];
  for (uint32_t li = 0; li < s->n_lanes; ++li) {
    o_run[li] = take(sizeof(JobDev) * (uint64_t)na);
    o_prep[li] = take(sizeof(JobDev) * (uint64_t)na);
    o_lim[li] = take(8ull * (na + 1));
    o_it[li] = take(8ull * (na + 1));
  }
  const uint64_t o_dg = take(8ull * D_COUNT);
  if (hipMalloc(&s->fixed_mem, o) != hipSuccess) { delete s; return CS_ENOMEM; }
  if (hipMalloc(&s->arena_mem, cfg->budget_bytes) != hipSuccess) {
    (void)hipFree(s->fixed_mem);
    delete s;
    return CS_ENOMEM;
  }
  s->arena.init(cfg->budget_bytes);
  uint8_t* m = s->fixed_mem;
  s->pw.n_base = reinterpret_cast<uint32_t*>(m + o_nb);
  s->pw.n_primes = reinterpret_cast<uint64_t*>(m + o_np);
  s->pw.base = reinterpret_cast<uint32_t*>(m + o_base);
  s->pw.flags = reinterpret_cast<uint32_t*>(m + o_fl);
  s->pw.seg_count = reinterpret_cast<uint32_t*>(m + o_sc);
  s->pw.seg_off = reinterpret_cast<uint64_t*>(m + o_so);
  s->pw.primes = reinterpret_cast<uint64_t*>(m + o_pr);
  s->pw.cap = cap;
  s->diag = reinterpret_cast<unsigned long long*>(m + o_dg);
  bool ok = true;
  for (uint32_t li = 0; li < s->n_lanes; ++li) {
    Lane& L = s->lane[li];
    L.run_dev = reinterpret_cast<JobDev*>(m + o_run[li]);
    L.prep_dev = reinterpret_cast<JobDev*>(m + o_prep[li]);
    L.lim_base = reinterpret_cast<uint64_t*>(m + o_lim[li]);
    L.items_base = reinterpret_cast<uint64_t*>(m + o_it[li]);
    ok = ok && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&L.aux, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&L.ev_fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&L.ev_join, hipEventDisableTiming) == hipSuccess;
  }
  // the resident prime table (the paper's one-time cost, Section 5)
  hipStream_t st0 = s->lane[0].stream;
  ok = ok && launch_primes(cfg->max_limit, s->pw, st0) == hipSuccess;
  ok = ok && launch_fill_u32(reinterpret_cast<uint32_t*>(s->diag), 2ull * D_COUNT, 0u, st0) == hipSuccess;
  ok = ok && hipStreamSynchronize(st0) == hipSuccess;
  if (!ok) {
    for (uint32_t li = 0; li < s->n_lanes; ++li) {
      Lane& L = s->lane[li];
      if (L.ev_fork) (void)hipEventDestroy(L.ev_fork);
      if (L.ev_join) (void)hipEventDestroy(L.ev_join);
      if (L.aux) (void)hipStreamDestroy(L.aux);
      if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    (void)hipFree(s->arena_mem);
    (void)hipFree(s->fixed_mem);
    delete s;
    return CS_EDEVICE;
  }
  for (uint32_t li = 0; li < s->n_lanes; ++li) s->lane[li].th = std::thread(server_loop, s, li);
  *out = s;
  return CS_OK;
}

extern "C" cs_status cs_server_submit(cs_server* s, const cs_job* job, uint64_t* ticket) {
  if (!s || !job || !ticket) return CS_EINVAL;
  Plan pl;
  cs_status st = plan_for_server(s, job, &pl);
  if (st) return st;
  if (job_bytes(pl) + (pl.kmod_fused ? 0 : kmod_bytes(job->limit)) + 512 > s->cfg.budget_bytes) return CS_ERANGE;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed) return CS_EDEVICE;
  const uint64_t t = s->next_ticket++;
  SJob& J = s->jobs[t];
  J.job = *job;
  J.plan = pl;
  J.t_submit = now_s();
  J.lane = (s->n_lanes > 1 && est_ms(pl) > s->cfg.long_ms) ? 1u : 0u;
  s->lane[J.lane].pending.push_back(t);
  s->st.submitted++;
  s->cv_work.notify_all();
  *ticket = t;
  return CS_OK;
}

extern "C" cs_status cs_server_poll(cs_server* s, uint64_t ticket, cs_ticket_info* out) {
  if (!s || !out) return CS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return CS_EINVAL;
  fill_info(s, it->second, out);
  return it->second.state == S_ERROR ? CS_EDEVICE : CS_OK;
}

extern "C" cs_status cs_server_wait(cs_server* s, uint64_t ticket, double timeout_s, cs_ticket_info* out) {
  if (!s) return CS_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return CS_EINVAL;
  const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  while (it->second.state == S_QUEUED || it->second.state == S_ACTIVE) {
    if (s->cv_done.wait_until(lk, until) == std::cv_status::timeout) break;
  }
  if (out) fill_info(s, it->second, out);
  if (it->second.state == S_ERROR) return CS_EDEVICE;
  return it->second.state == S_DONE ? CS_OK : CS_EBUSY;
}

extern "C" cs_status cs_server_copy_outputs(cs_server* s, uint64_t ticket, uint32_t* d_bitmap, uint32_t* d_counts,
                                            void* stream) {
  if (!s) return CS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return CS_EINVAL;
  SJob& J = it->second;
  if (J.state == S_ERROR) return CS_EDEVICE;
  if (J.state != S_DONE) return CS_EBUSY;
  const uint64_t bb = J.plan.n_m * (uint64_t)J.plan.row_words * 4ull, cb = J.plan.n_m * 4ull;
  if (J.plan.n_m == 0) return CS_OK;
  if (!d_bitmap || !d_counts) return CS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(d_bitmap, J.jd.bitmap, bb, hipMemcpyDeviceToDevice, st) != hipSuccess) return CS_EDEVICE;
  if (hipMemcpyAsync(d_counts, J.jd.counts, cb, hipMemcpyDeviceToDevice, st) != hipSuccess) return CS_EDEVICE;
  return CS_OK;
}

extern "C" cs_status cs_server_release(cs_server* s, uint64_t ticket) {
  if (!s) return CS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return CS_EINVAL;
  SJob& J = it->second;
  if (J.state == S_QUEUED || J.state == S_ACTIVE) return CS_EBUSY;
  if (J.bytes_out) s->arena.release(J.off_out, J.bytes_out);
  s->jobs.erase(it);
  return CS_OK;
}

extern "C" cs_status cs_server_stats(cs_server* s, cs_server_counters* out) {
  if (!s || !out) return CS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->bytes_in_use = s->arena.used();
  out->active = 0;
  out->queued = 0;
  for (uint32_t li = 0; li < s->n_lanes; ++li) {
    out->active += s->lane[li].active.size();
    out->queued += s->lane[li].pending.size();
  }
  return s->failed ? CS_EDEVICE : CS_OK;
}

extern "C" cs_status cs_server_destroy(cs_server* s) {
  if (!s) return CS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  for (uint32_t li = 0; li < s->n_lanes; ++li) {
    Lane& L = s->lane[li];
    if (L.th.joinable()) L.th.join();
    (void)hipStreamSynchronize(L.stream);
    (void)hipStreamSynchronize(L.aux);
    (void)hipEventDestroy(L.ev_fork);
    (void)hipEventDestroy(L.ev_join);
    (void)hipStreamDestroy(L.aux);
    (void)hipStreamDestroy(L.stream);
  }
  (void)hipFree(s->arena_mem);
  (void)hipFree(s->fixed_mem);
  delete s;
  return CS_OK;
}

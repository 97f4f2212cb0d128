// Host-side planning for the Combined Sieve library.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "plan.h"

namespace cs {

typedef unsigned __int128 u128;

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

uint64_t pi_upper(uint64_t x) {
  if (x < 17) return 7;
  const double lx = log((double)x);
  double b;
  if (x >= 355991) b = (double)x / lx * (1.0 + 1.0 / lx + 2.51 / (lx * lx));   // Dusart 2010
  else b = 1.25506 * (double)x / lx;                                            // Rosser-Schoenfeld
  return (uint64_t)b + 64;
}

// Default small/large threshold of the three-gap walk, from the two branches' costs: a small
// prime costs about n_m residue steps of c_pair = 0.83 ps, a large prime about n_m n_x / p hit
// atomics of c_hit = 55 ps.  Where the hits take long (over 40 ms), the small branch runs hidden
// beside them on its own stream while it takes at most about two fifths of their time: the
// largest C_mult of 30, 36, 44, 52 and 64 that keeps it there (at 953#/210, m_inc 1e6, limit 1e10
// that is 52: one call 79.6 ms, against 84.4 ms at 30 S, 80.9 at 44 S and 83.4 at 64 S; with
// limit 1e9 it is 36, within 2% of the best multiple measured there).  Otherwise the
// two branches' times add, and the sum n_m pi(thr) c_pair' + n_m n_x (log log limit - log log thr)
// c_hit is least at thr = n_x c_hit / c_pair' = 44 n_x, with c_pair' = 1.25 ps measured for jobs
// of fewer rows (96 mixed jobs alone: 307 ms in all, against 361 ms at 30 S).
static uint64_t three_gap_threshold(const cs_job& j, const Plan& pl) {
  constexpr double kPair = 0.83e-12, kHit = 55e-12;
  const double L = std::max<double>((double)j.limit, 16.0);
  auto pi_est = [](double x) { return x / (log(x) - 1.0); };
  auto hit_s = [&](double t) {
    return (double)pl.n_m * pl.n_x * std::max(0.0, log(log(L)) - log(log(std::max(t, 3.0)))) * kHit;
  };
  uint64_t thr = 44ull * std::max<uint32_t>(pl.n_x, 1u);
  const double t30 = 30.0 * (double)pl.S;
  if (t30 < L && hit_s(t30) > 40e-3) {
    thr = (uint64_t)t30;
    for (double cm : {36.0, 44.0, 52.0, 64.0}) {
      const double t = cm * (double)pl.S;
      if (t >= L || (double)pl.n_m * pi_est(t) * kPair > 0.4 * hit_s(t)) break;
      thr = (uint64_t)t;
    }
  }
  return thr;
}

static std::vector<uint32_t> host_primes_upto(uint32_t n) {
  std::vector<uint8_t> comp(n + 1, 0);
  std::vector<uint32_t> out;
  for (uint64_t i = 2; i <= n; ++i) {
    if (comp[i]) continue;
    out.push_back((uint32_t)i);
    for (uint64_t j = i * i; j <= n; j += i) comp[j] = 1;
  }
  return out;
}

void host_columns(const cs_job& job, const std::vector<uint32_t>& kq, std::vector<int32_t>* xs) {
  const uint32_t sl = job.sl;
  std::vector<uint8_t> bad(2 * (size_t)sl + 1, 0);
  for (uint32_t q : kq) {
    if (q > sl) break;
    for (uint64_t x = q; x <= sl; x += q) {
      bad[sl + x] = 1;
      bad[sl - x] = 1;
    }
  }
  if (!kq.empty()) bad[sl] = 1;    // gcd(0, K) = K > 1
  xs->clear();
  for (uint64_t i = 0; i < bad.size(); ++i)
    if (!bad[i]) xs->push_back((int32_t)((int64_t)i - (int64_t)sl));
}

// #{m in [0, x) : gcd(m, d) = 1} by inclusion-exclusion over the prime factors of d.
static u128 coprime_below(u128 x, const std::vector<uint32_t>& dq) {
  const size_t k = dq.size();
  u128 acc_pos = 0, acc_neg = 0;
  for (uint64_t mask = 0; mask < (1ull << k); ++mask) {
    u128 e = 1;
    int bits = 0;
    for (size_t t = 0; t < k; ++t)
      if (mask >> t & 1) { e *= dq[t]; ++bits; }
    const u128 c = (x + e - 1) / e;
    if (bits & 1) acc_neg += c; else acc_pos += c;
  }
  return acc_pos - acc_neg;
}

uint64_t host_row_count(const cs_job& job, const std::vector<uint32_t>& dq) {
  return (uint64_t)(coprime_below((u128)job.m_start + job.m_inc, dq) - coprime_below(job.m_start, dq));
}

cs_status make_plan(const cs_job* job, const cs_tune* tune, int n_cu, Plan* out, bool own_primes, bool own_kmod,
                    bool bytes_ok, uint64_t span) {
  if (!job || !out) return CS_EINVAL;
  const cs_job j = *job;
  if (j.P < 2 || j.P >= kMaxP) return CS_EINVAL;
  if (j.d == 0 || j.m_start == 0 || j.m_inc == 0) return CS_EINVAL;
  if (j.m_inc >= kMaxMInc) return CS_EINVAL;
  if (j.m_start >= (1ull << 63) || j.m_inc >= (1ull << 63) - j.m_start) return CS_EINVAL;
  if (j.sl == 0 || j.sl > kMaxSl) return CS_EINVAL;
  if (j.limit < 2) return CS_EINVAL;
  if (j.limit >= kMaxLimit) return CS_ERANGE;
  const uint32_t mode = tune ? tune->large_mode : CS_LARGE_G;
  if (mode > CS_LARGE_THREE_GAP) return CS_EINVAL;
  const uint32_t scatter = tune ? tune->scatter : CS_SCATTER_AUTO;
  if (scatter > CS_SCATTER_LIST) return CS_EINVAL;
  if (tune && tune->walk > CS_WALK_ALL) return CS_EINVAL;
  if (tune && tune->wide_log2 && (tune->wide_log2 < 20 || tune->wide_log2 > 42)) return CS_EINVAL;
  if (tune && tune->kmod > CS_KMOD_TABLE) return CS_EINVAL;

  Plan& pl = *out;
  pl.job = j;
  pl.kq.clear();
  pl.dq.clear();
  std::vector<uint32_t> ps = host_primes_upto(j.P);
  uint64_t rest = j.d;
  for (uint32_t q : ps) {
    if (rest % q == 0) {
      rest /= q;
      if (rest % q == 0) return CS_EINVAL;    // not squarefree
      pl.dq.push_back(q);
    } else {
      pl.kq.push_back(q);
    }
  }
  if (rest != 1) return CS_EINVAL;            // d does not divide P#
  if (pl.dq.size() > (size_t)kMaxDq) return CS_EINVAL;
  // every N + X must be positive: sl < m_start * K
  {
    u128 K = 1;
    bool big = false;
    for (uint32_t q : pl.kq) {
      K *= q;
      if (K >> 64) { big = true; break; }
    }
    if (!big && (u128)j.sl >= K * (u128)j.m_start) return CS_EINVAL;
  }

  pl.Lp = std::max<uint64_t>(j.limit, j.P);
  pl.span = 0;
  if (span) {
    // chunks of the prime range: segment-aligned, and the first one holds every prime <= P
    if (span % kSpanAlign || span < kMinSpan || span <= j.P) return CS_EINVAL;
    if (span < pl.Lp + 1) {
      pl.span = span;
      pl.Lp = span - 1;
    }
  }
  pl.n_seg = (pl.Lp >> kSegLog) + 1;
  // A chunk [x, x + span) holds no more primes than [0, span) in practice; a denser chunk would
  // be reported (E_PRIMES), never written past the table.
  pl.cap = pi_upper(pl.Lp) + (pl.span ? 1024 : 0);
  pl.n_m = host_row_count(j, pl.dq);
  std::vector<int32_t> xs;
  host_columns(j, pl.kq, &xs);
  pl.n_x = (uint32_t)xs.size();
  pl.row_words = (pl.n_x + 31) / 32;
  pl.S = 2 * j.sl + 1;
  pl.ct_words = (pl.S + 31) / 32;
  pl.w = 2 * j.sl;
  pl.large_mode = mode;
  pl.walk_all = tune && tune->walk == CS_WALK_ALL;
  pl.wide_lo = tune && tune->wide_log2 ? (1ull << tune->wide_log2) : kWideLo;

  // small/large threshold C_mult * S (Section 5).  With one Eq. 5 solve per hit, C_mult =
  // 2.5 M / M_c (a quarter of the paper's 10 M / M_c: at 953#/210 the step is flat from 120,000
  // to 437,507 = 2.5 M / M_c S, 216-218 ms, against 223 ms at 5 M / M_c S).  With three-gap
  // stepping the threshold comes from the two branches' costs (three_gap_threshold).  Clamped so
  // that a large prime divides at most one number of an interval (p > 2 sl), or (three-gap) p > 4 sl.
  uint64_t thr_min = std::max<uint64_t>(j.P, pl.w);
  if (mode == CS_LARGE_THREE_GAP) thr_min = std::max<uint64_t>(thr_min, 2ull * pl.w);
  uint64_t thr = tune && tune->thr ? tune->thr : 0;
  if (!thr) {
    if (mode == CS_LARGE_THREE_GAP) {
      thr = three_gap_threshold(j, pl);
    } else {
      const double cm = pl.n_m ? 2.5 * (double)j.m_inc / (double)pl.n_m : 2.5;
      thr = (uint64_t)(cm * (double)pl.S);
    }
  }
  pl.thr = std::max(thr, thr_min);
  // the small branch and the fp64 large branch stop below wide_lo
  if (thr_min >= pl.wide_lo) return CS_EINVAL;
  pl.thr = std::min<uint64_t>(pl.thr, pl.wide_lo - 1);
  // the small branch's hit-row pass where most small primes lie far above w (it pays at the paper
  // scale, 52 S = 52 w; on the mixed jobs, whose thresholds sit at 4-18 w, the instance without it
  // ran faster)
  pl.small_hit_rows = pl.thr >= 24ull * std::max<uint64_t>(pl.w, 1);

  // small branch tiles
  const bool ct_lds = pl.ct_words * 8u <= kLdsCtMax;
  const uint32_t ct_bytes = ct_lds ? pl.ct_words * 8u : 0u;
  uint32_t rows = (kLdsBudget - ct_bytes) / (4u * pl.row_words + 8u);
  rows = std::max(1u, std::min(rows, kTileRowsMax));
  if (tune && tune->tile_rows) rows = std::min(rows, tune->tile_rows);
  pl.tile_rows = rows;
  pl.n_windows = (uint32_t)((pl.n_m + rows - 1) / rows);
  pl.lds_ct_words = ct_lds ? pl.ct_words : 0;
  pl.lds_bytes = ct_bytes + 4u * rows * pl.row_words + 8u * rows;   // tile, counts, m offsets
  const double est_small = (double)pl.thr / std::max(1.0, log((double)pl.thr));
  // prime slices per row window (at least 512 primes each) so that a job of few windows still
  // fills the GPU: up to 4 workgroups per CU in all
  uint32_t max_slices = (uint32_t)std::max(1.0, std::min(4096.0, est_small / 512.0));
  uint32_t slices = pl.n_windows ? (uint32_t)((4u * (uint32_t)n_cu + pl.n_windows - 1) / pl.n_windows) : 1;
  slices = std::max(1u, std::min(slices, max_slices));
  if (tune && tune->small_slices) slices = std::min(tune->small_slices, 256u);
  pl.n_slices = slices;
  const uint64_t units = (uint64_t)pl.n_windows * slices;
  pl.small_blocks = (uint32_t)std::min<uint64_t>(units ? units : 1, 1ull << 31);   // one workgroup per unit
  pl.dense_max = std::max<uint64_t>(1, pl.w / 32);

  // residue table of d: m -> row without a per-m lookup
  pl.dpre.clear();
  pl.phi_d = 0;
  pl.r0_d = 0;
  if (j.d <= kDSmall) {
    const uint32_t d32 = (uint32_t)j.d;
    pl.dpre.resize(d32);
    uint32_t c = 0;
    for (uint32_t r = 0; r < d32; ++r) {
      bool cop = true;
      for (uint32_t q : pl.dq)
        if (r % q == 0) { cop = false; break; }
      if (d32 == 1) cop = true;
      pl.dpre[r] = (uint16_t)(c | (cop ? 0x8000u : 0u));
      c += cop ? 1 : 0;
    }
    pl.phi_d = c;
    pl.r0_d = (uint32_t)(j.m_start % j.d);
    pl.dres.clear();
    for (uint32_t r = 0; r < d32; ++r)
      if (pl.dpre[r] & 0x8000u) pl.dres.push_back((uint16_t)r);
  }
  pl.dpat_on = !pl.dpre.empty() && j.d > 1 && pl.n_m > 0 &&
               (uint64_t)pl.phi_d * pl.row_words * 4ull <= (64ull << 20);
  {
    const uint32_t ct_b = pl.ct_words * 8u;
    const uint32_t dp_b = (uint32_t)pl.dpre.size() * 2u;
    pl.large_lds_ct_words = ct_b <= 16384u ? pl.ct_words : 0u;
    pl.large_lds_bytes = (pl.large_lds_ct_words ? ct_b : 0u) + ((dp_b + 3u) & ~3u);
    // K mod p formed in the large branch: a job with its own K mod p table (a single job, or one of
    // a batch or a server), no chunks and no prime on the 64-bit path; K's groups (at most one per
    // prime dividing K) as doubles in its LDS
    pl.kmod_fused = own_kmod && span == 0 &&
                    (!tune || tune->kmod == CS_KMOD_AUTO) && std::max<uint64_t>(j.limit, j.P) < pl.wide_lo &&
                    pl.kq.size() <= kFusedGroupsMax;
    pl.kg_lds_off = 0;
    if (pl.kmod_fused && pl.large_lds_ct_words) {
      pl.kg_lds_off = (pl.large_lds_bytes + 7u) & ~7u;
      pl.large_lds_bytes = pl.kg_lds_off + 8u * (uint32_t)std::max<size_t>(pl.kq.size(), 1);
    }
  }

  pl.hits_per_item = tune && tune->hits_per_item ? tune->hits_per_item
                                                 : (mode == CS_LARGE_G ? 128u : 1024u);

  // workspace layout
  WsLayout& L = pl.ws;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) { uint64_t at = o; o = align256(o + std::max<uint64_t>(bytes, 8)); return at; };
  const uint64_t cap_lim = pl.span ? pl.cap : pi_upper(j.limit);
  // Limits from 2^42 on need base primes beyond the two LDS windows of k_base_primes (2^21): the
  // primes up to the square root of the limit are sieved first into their own table.
  pl.isq = 0;
  const uint64_t top = std::max<uint64_t>(j.limit, j.P);
  if (own_primes && top >= kWideLo) {
    uint64_t r = (uint64_t)sqrtl((long double)top);
    while (r * r > top) --r;
    while ((r + 1) * (r + 1) <= top) ++r;
    pl.isq = r;
    pl.n_seg2 = (r >> kSegLog) + 1;
    pl.cap2 = pi_upper(r);
  }

  L.ctrl = take(sizeof(JobCtrl));
  L.jobdev = take(sizeof(JobDev));
  L.items_base = take(2 * sizeof(uint64_t));
  L.lim_base = take(2 * sizeof(uint64_t));
  L.n_base = take(8);
  L.n_primes = take(8);
  const uint64_t ns = own_primes ? pl.n_seg : 0;
  L.base = take(own_primes ? kBaseCap * 4ull : 0);
  L.flags = take(ns * kSegWords * 4ull);
  L.seg_count = take(ns * 4ull);
  L.seg_off = take(ns * 8ull);
  L.primes = take(own_primes ? pl.cap * 8ull : 0);
  // with K mod p formed in the large branch the tables hold the primes <= thr only
  const uint64_t cap_km = pl.kmod_fused ? std::min<uint64_t>(cap_lim, pi_upper(pl.thr)) : cap_lim;
  L.kmod = take(own_kmod ? cap_km * 8ull : 0);
  L.mk = take(cap_km * 8ull);
  L.row_of = take(j.m_inc * 4ull);
  L.m_off = take(std::max<uint64_t>(pl.n_m, 1) * 4ull);
  L.row_blk = take(((j.m_inc + 1023) / 1024) * 4ull);
  L.coltab = take(pl.ct_words * 8ull);
  L.kgroups = take((pl.kq.size() + 1) * 8ull);
  L.kq = take((pl.kq.size() + 1) * 4ull);
  L.dpre = take(std::max<uint64_t>(pl.dpre.size(), 1) * 2ull);
  L.dres = take(std::max<uint64_t>(pl.dres.size(), 1) * 2ull);
  L.dpat = take(pl.dpat_on ? (uint64_t)pl.phi_d * pl.row_words * 4ull : 0);
  L.dpat_cnt = take(pl.dpat_on ? (uint64_t)pl.phi_d * 4ull : 0);
  // Byte counters are exact when no number m K + X of the interval has 256 or more distinct prime
  // factors above the threshold: their product exceeds thr^c, and m K + X < (m_start + m_inc) K.
  {
    double log2_n = log2((double)j.m_start + (double)j.m_inc + 1.0);
    for (uint32_t q : pl.kq) log2_n += log2((double)q);
    const double c_max = floor(log2_n * (1.0 + 1e-12) / log2((double)pl.thr + 1.0));
    pl.cell_max = c_max;
    const bool fits = c_max < 256.0;
    if (scatter == CS_SCATTER_BYTES && !fits) return CS_EINVAL;
    // List scatter: a pool of about 1.15x the expected large hits, n_m n_x times the sum of 1/p
    // over the large primes (log log limit - log log thr by Mertens), plus one open chunk per
    // wavefront of the large-branch grid.
    // Cells are (row << cell_shift) | col; buckets hold 2^k rows whose LDS tile fits
    // kListTileBytes (at most 64 rows); groups hold 2^g buckets, at most kListSupers groups.
    pl.scatter_list = false;
    pl.list_chunks = 0;
    // every wavefront of the large branch may leave one chunk part-filled: the list keeps a
    // smaller grid than the default
    const uint32_t list_blocks = tune && tune->large_blocks ? tune->large_blocks : (uint32_t)n_cu * kListBlocksPerCu;
    pl.cell_shift = 0;
    while ((1ull << pl.cell_shift) < std::max<uint64_t>(pl.n_x, 1)) ++pl.cell_shift;
    uint32_t lb = 0;
    while (lb < 6 && (2ull << lb) * (pl.row_words * 4ull + 4ull) <= kListTileBytes) ++lb;
    pl.bkt_rows = 1u << lb;
    pl.n_bkt = (uint32_t)std::min<uint64_t>((pl.n_m + pl.bkt_rows - 1) >> lb, 0xffffffffull);
    pl.super_shift = 0;
    while (((uint64_t)pl.n_bkt + (1ull << pl.super_shift) - 1) >> pl.super_shift > kListSupers) ++pl.super_shift;
    {
      const double sum_inv = j.limit > pl.thr + 1 ? std::max(0.0, log(log((double)j.limit)) - log(log((double)pl.thr + 1.0)))
                                                  : 0.0;
      const double expect = (double)pl.n_m * (double)pl.n_x * sum_inv;
      const uint64_t slack = std::max<uint64_t>(list_blocks, 2048) * 4ull + 4ull;   // open chunks
      const uint64_t chunks = (uint64_t)(expect * 1.15 / kListChunk) + slack;
      const bool ok = own_primes && pl.n_m > 0 && (pl.n_m << pl.cell_shift) <= (1ull << 32) &&
                      pl.n_bkt <= kMaxBuckets && (1u << pl.super_shift) <= kListMaxPerSuper &&
                      (double)chunks * kListChunk < 4294967296.0;
      if (scatter == CS_SCATTER_LIST && !ok) return CS_EINVAL;
      // AUTO does not take the list: its grouping passes cost more than the atomics they remove
      // (measured at the paper scale: large-prime kernel 53 ms plus 35 ms of grouping with the
      // list, and a step of 153 ms without the small branch alongside, against 84 ms and a
      // 101 ms step with the byte counters).
      if (ok && scatter == CS_SCATTER_LIST) {
        pl.scatter_list = true;
        pl.list_chunks = tune && tune->list_chunks ? std::min<uint64_t>(tune->list_chunks, chunks) : chunks;
      }
    }
    pl.scatter_bytes = !pl.scatter_list && bytes_ok && fits &&
                       (scatter == CS_SCATTER_AUTO || scatter == CS_SCATTER_BYTES);
    pl.large_blocks = pl.scatter_list ? list_blocks
                    : tune && tune->large_blocks ? tune->large_blocks : (uint32_t)n_cu * kLargeBlocksPerCu;
  }
  L.hitbytes = take(pl.scatter_bytes ? pl.n_m * (uint64_t)pl.row_words * 32ull : 0);
  L.list_pool = take(pl.list_chunks * kListChunk * 4ull);
  L.list_fill = take(pl.list_chunks * 4ull);
  L.list_cursor = take(8);
  L.list_sorted = take(pl.list_chunks * kListChunk * 4ull);
  L.bkt_count = take(pl.scatter_list ? (pl.n_bkt + 1ull) * 4ull : 0);
  L.bkt_base = take(pl.scatter_list ? (pl.n_bkt + 1ull) * 4ull : 0);
  L.bkt_cursor = take(pl.scatter_list ? (pl.n_bkt + 1ull) * 4ull : 0);
  L.list_super = take(pl.scatter_list ? 3ull * (kListSupers + 1) * 4ull : 0);
  // (the control block stays at offset 0: cs_diag_read reads it there)
  L.base2 = take(pl.isq ? pl.cap2 * 8ull : 0);
  L.n_base2 = take(8);
  L.flags2 = take(pl.isq ? pl.n_seg2 * kSegWords * 4ull : 0);
  L.seg_count2 = take(pl.isq ? pl.n_seg2 * 4ull : 0);
  L.seg_off2 = take(pl.isq ? pl.n_seg2 * 8ull : 0);
  L.total = o;
  return CS_OK;
}

void walk_classes(const Plan& pl, uint32_t* step, uint32_t* classes) {
  // Only m coprime to d are rows.  Walking one class mod s costs one first solve per item and
  // class, and visits 1/s of the m: with one solve per hit every visited m costs a solve, so the
  // classes mod 6 pay when 6 | d (1/3 of the m for two first solves); three-gap stepping takes a
  // few operations per visited m and keeps the single class mod 2.
  const uint64_t d = pl.job.d;
  if (pl.walk_all) {
    *step = 1;
    *classes = 1u;
  } else if (pl.large_mode == CS_LARGE_G && d % 6 == 0) {
    *step = 6;
    *classes = (1u << 1) | (1u << 5);
  } else if (d % 2 == 0) {
    *step = 2;
    *classes = 1u << 1;
  } else {
    *step = 1;
    *classes = 1u;
  }
}

void fill_tiers(const Plan& pl, uint64_t p_lo, uint64_t p_hi, JobDev* jd) {
  const uint64_t lo = std::max<uint64_t>(pl.thr, p_lo > 0 ? p_lo - 1 : 0);
  const uint64_t hi = std::min<uint64_t>(p_hi, pl.job.limit);
  jd->dpat_apply = (pl.dpat_on && !pl.dq.empty() && p_lo <= pl.dq.front() &&
                    (uint64_t)pl.dq.back() <= std::min<uint64_t>(p_hi, pl.job.limit)) ? 1u : 0u;
  jd->tier_lo = lo;
  jd->n_tiers = 0;
  if (hi <= lo || pl.n_m == 0) return;
  // positions the large branch visits per prime: the m of its residue classes
  uint32_t step = 1, classes = 1;
  walk_classes(pl, &step, &classes);
  const double walked = ceil((double)pl.job.m_inc / step) * __builtin_popcount(classes);
  const double mw = walked * (double)(pl.w + 1);
  const double H = (double)pl.hits_per_item;
  uint64_t b = lo;
  uint32_t nt = 0;
  while (b < hi) {
    uint64_t nb = std::min<uint64_t>(hi, std::max<uint64_t>(2 * b, b + 1));
    double expect = mw / (double)(b + 1);
    uint64_t C = (uint64_t)ceil(expect / H);
    C = std::max<uint64_t>(1, std::min<uint64_t>(C, pl.job.m_inc));
    C = std::min<uint64_t>(C, 1u << 30);
    if (nt > 0 && jd->tier_chunks[nt - 1] == (uint32_t)C) {
      jd->tier_hi[nt - 1] = nb;
    } else if (nt < (uint32_t)kMaxTiers) {
      jd->tier_hi[nt] = nb;
      jd->tier_chunks[nt] = (uint32_t)C;
      ++nt;
    } else {
      jd->tier_hi[nt - 1] = nb;      // more chunks than needed is still exact
      jd->tier_chunks[nt - 1] = std::max<uint32_t>(jd->tier_chunks[nt - 1], (uint32_t)C);
    }
    b = nb;
  }
  jd->n_tiers = nt;
}

JobDev make_jobdev(const Plan& pl, uint8_t* ws, const uint64_t* primes, const uint64_t* n_primes) {
  JobDev jd;
  memset(&jd, 0, sizeof(jd));
  const cs_job& j = pl.job;
  jd.d = j.d;
  jd.m_start = j.m_start;
  jd.m_inc = j.m_inc;
  walk_classes(pl, &jd.m_step, &jd.m_classes);
  jd.m0_mod_step = (uint32_t)(j.m_start % jd.m_step);
  jd.limit = j.limit;
  jd.thr = pl.thr;
  jd.p_lo = 2;
  jd.p_hi = j.limit;
  jd.n_m = pl.n_m;
  jd.P = j.P;
  jd.sl = j.sl;
  jd.w = pl.w;
  jd.n_x = pl.n_x;
  jd.row_words = pl.row_words;
  jd.large_mode = pl.large_mode;
  jd.tile_rows = pl.tile_rows;
  jd.n_windows = pl.n_windows;
  jd.n_slices = pl.n_slices;
  jd.hits_per_item = pl.hits_per_item;
  jd.small_unit_base = 0;
  jd.dense_max = pl.dense_max;
  jd.prime_cap = pl.cap;
  jd.wide_lo = pl.wide_lo;
  jd.kmod_fused = pl.kmod_fused ? 1u : 0u;
  jd.primes = primes;
  jd.n_primes = n_primes;
  const WsLayout& L = pl.ws;
  jd.kmod = reinterpret_cast<uint64_t*>(ws + L.kmod);
  jd.mk = reinterpret_cast<uint64_t*>(ws + L.mk);
  jd.row_of = reinterpret_cast<int32_t*>(ws + L.row_of);
  jd.m_off = reinterpret_cast<uint32_t*>(ws + L.m_off);
  jd.row_blk = reinterpret_cast<uint32_t*>(ws + L.row_blk);
  jd.coltab = reinterpret_cast<uint2*>(ws + L.coltab);
  jd.kgroups = reinterpret_cast<uint64_t*>(ws + L.kgroups);
  jd.kq = reinterpret_cast<uint32_t*>(ws + L.kq);
  jd.ctrl = reinterpret_cast<JobCtrl*>(ws + L.ctrl);
  jd.d_small = pl.dpre.empty() ? 0u : 1u;
  jd.phi_d = pl.phi_d;
  jd.r0_d = pl.r0_d;
  jd.pre_r0 = pl.dpre.empty() ? 0u : (uint32_t)(pl.dpre[pl.r0_d] & 0x7fffu);
  jd.inv_d = 1.0 / (double)j.d;
  jd.dpre = reinterpret_cast<const uint16_t*>(ws + L.dpre);
  jd.dres = reinterpret_cast<const uint16_t*>(ws + L.dres);
  jd.dpat_on = pl.dpat_on ? 1u : 0u;
  jd.dpat = reinterpret_cast<uint32_t*>(ws + L.dpat);
  jd.dpat_cnt = reinterpret_cast<uint32_t*>(ws + L.dpat_cnt);
  jd.hitbytes = pl.scatter_bytes ? ws + L.hitbytes : nullptr;
  jd.list_pool = pl.scatter_list ? reinterpret_cast<uint32_t*>(ws + L.list_pool) : nullptr;
  jd.list_fill = reinterpret_cast<uint32_t*>(ws + L.list_fill);
  jd.list_cursor = reinterpret_cast<unsigned long long*>(ws + L.list_cursor);
  jd.list_sorted = reinterpret_cast<uint32_t*>(ws + L.list_sorted);
  jd.bkt_count = reinterpret_cast<uint32_t*>(ws + L.bkt_count);
  jd.bkt_base = reinterpret_cast<uint32_t*>(ws + L.bkt_base);
  jd.bkt_cursor = reinterpret_cast<uint32_t*>(ws + L.bkt_cursor);
  jd.list_super = reinterpret_cast<uint32_t*>(ws + L.list_super);
  jd.list_chunks = pl.list_chunks;
  jd.n_bkt = pl.n_bkt;
  jd.bkt_rows = pl.bkt_rows;
  jd.bkt_per_super = 1u << pl.super_shift;
  jd.cell_shift = pl.cell_shift;
  jd.bkt_shift = pl.cell_shift + (uint32_t)__builtin_ctz(pl.bkt_rows);
  jd.super_shift = pl.super_shift;
  fill_tiers(pl, 2, j.limit, &jd);
  return jd;
}

int device_cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

}  // namespace cs

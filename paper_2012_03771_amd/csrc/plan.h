// Host-side job planning: validation, row/column counts, workspace layout, work decomposition.
#pragma once
#include <stdint.h>
#include <vector>

#include "../../include/csieve.h"
#include "device.h"

namespace cs {

constexpr uint32_t kMaxSl = (1u << 17) - 1;     // a packed row (<= 2^18 bits) fits an LDS tile
constexpr uint64_t kMaxLimit = 1ull << 63;    // sieve limits of single jobs (chunked beyond memory)
constexpr uint64_t kWideLo = 1ull << 42;      // primes from here take the exact 64-bit residue path;
                                              // batches, the server and cs_primes stay below it
constexpr uint32_t kMaxP = 1u << 24;
constexpr uint64_t kMaxMInc = 1ull << 32;
constexpr uint32_t kSmallBlock = 512;
constexpr uint32_t kLargeBlock = 256;
// Default grid of the large branch: many short workgroups, so the hardware scheduler evens out
// the items' unequal costs (a persistent grid of a few workgroups per CU left a long tail).
constexpr uint32_t kLargeBlocksPerCu = 128;
constexpr uint32_t kListBlocksPerCu = 8;      // with the list scatter (one part-filled chunk per wavefront)
constexpr uint32_t kLdsBudget = 64 * 1024 - 256;   // dynamic LDS of a small-branch tile (the kernel keeps 256 B of its own)
constexpr uint32_t kLdsCtMax = 32 * 1024;
constexpr uint32_t kTileRowsMax = 16;          // rows per small-branch tile (more workgroups per CU beat bigger tiles)
constexpr uint32_t kBaseCap = 155700;           // odd primes below 2^21 (155,610) plus slack

struct WsLayout {
  uint64_t ctrl;                     // always 0: cs_diag_read reads the control block there
  uint64_t base2, n_base2, flags2, seg_count2, seg_off2;   // level-2 base primes (limits >= 2^42)
  uint64_t jobdev, items_base, lim_base, base, n_base, n_primes, flags, seg_count, seg_off, primes,
      kmod, mk, row_of, m_off, row_blk, coltab, kgroups, kq, dpre, dres, dpat, dpat_cnt, hitbytes, list_pool,
      list_fill, list_cursor, list_sorted, bkt_count, bkt_base, bkt_cursor, list_super, total;
};

struct Plan {
  cs_job job;
  uint64_t Lp;              // max(limit, P): extent of the prime table (one chunk when span > 0)
  uint64_t span;            // chunked sieve: integers per chunk of the prime range; 0 = whole range
  uint64_t n_seg;
  uint64_t cap;             // prime table capacity
  uint64_t n_m;
  uint32_t n_x, row_words, S, ct_words;
  uint32_t w;
  uint64_t thr;
  uint32_t large_mode;
  bool walk_all = false;            // the large branch visits every m (CS_WALK_ALL)
  uint64_t wide_lo = kWideLo;       // primes >= wide_lo take the 64-bit residue path
  uint64_t isq = 0, cap2 = 0, n_seg2 = 0;   // level-2 base primes: up to isq (0: not needed)
  uint32_t tile_rows, n_windows, n_slices;
  uint32_t hits_per_item;
  uint32_t large_blocks, small_blocks;
  bool small_hit_rows = false;      // k_small with the hit-row pass (thr >= 24 w)
  uint32_t lds_bytes, lds_ct_words;
  uint32_t large_lds_bytes, large_lds_ct_words;   // LDS tables of the large branch (0: global)
  uint64_t dense_max;
  uint32_t phi_d, r0_d;
  std::vector<uint16_t> dpre;       // residue table when d <= kDSmall
  std::vector<uint16_t> dres;       // residues coprime to d (d <= kDSmall)
  bool dpat_on = false;             // per-class pattern of the primes dividing d
  bool scatter_bytes = false;       // large hits via byte counters (see CS_SCATTER_BYTES)
  double cell_max = 0;              // bound on large-prime hits of one (row, column)
  bool scatter_list = false;        // large hits via the list scatter (see CS_SCATTER_LIST)
  bool kmod_fused = false;          // the large branch forms K mod p itself; the table stops at thr
  uint32_t kg_lds_off = 0;          // large-branch LDS: byte offset of the K groups (fused, LDS tables)
  uint64_t list_chunks = 0;         // pool capacity in chunks
  uint32_t n_bkt = 0, bkt_rows = 0; // row buckets of the list scatter (bkt_rows a power of two)
  uint32_t cell_shift = 0, super_shift = 0;
  std::vector<uint32_t> kq;         // primes dividing K
  std::vector<uint32_t> dq;         // primes dividing d
  WsLayout ws;
};

// Upper bound of pi(x).
uint64_t pi_upper(uint64_t x);

// Validates the job and fills everything except the range-dependent tiers.  With own_primes
// false the workspace layout leaves out the prime table (a batch or server shares one); with
// own_kmod false it leaves out the K mod p table (a server shares one per (P, d)); with bytes_ok
// false the large-hit byte counters are not used (the server, which folds nothing).
cs_status make_plan(const cs_job* job, const cs_tune* tune, int n_cu, Plan* out, bool own_primes = true,
                    bool own_kmod = true, bool bytes_ok = true, uint64_t span = 0);
// Smallest and largest chunk of the prime range accepted by the chunked sieve (integers).
constexpr uint64_t kMinSpan = 1ull << 25;
constexpr uint64_t kSpanAlign = 1ull << 19;   // one prime-sieve segment

// Host count of rows and columns (also used by cs_rows / cs_columns).
void host_columns(const cs_job& job, const std::vector<uint32_t>& kq, std::vector<int32_t>* xs);
uint64_t host_row_count(const cs_job& job, const std::vector<uint32_t>& dq);

// Fills the range-dependent part of a job descriptor (tiers for primes in (max(thr, p_lo-1), p_hi]).
void fill_tiers(const Plan& pl, uint64_t p_lo, uint64_t p_hi, JobDev* jd);
// Residue classes of m the large branch walks: stride *step (dividing d) and the bit mask of the
// classes coprime to it.
void walk_classes(const Plan& pl, uint32_t* step, uint32_t* classes);

// Job descriptor with pointers into a workspace at `ws` (outputs left null).
JobDev make_jobdev(const Plan& pl, uint8_t* ws, const uint64_t* primes, const uint64_t* n_primes);

int device_cu_count();

}  // namespace cs

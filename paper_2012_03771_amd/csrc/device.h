// Device-side job descriptors shared by the kernels and the host launch code.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace cs {

constexpr int kMaxTiers = 48;     // large-branch prime tiers (chunk count per tier)
constexpr int kMaxDq = 16;        // prime factors of d (d < 2^64 squarefree has at most 15)
constexpr int kSegLog = 19;       // prime sieve segment: 2^19 integers, odd-only bits
constexpr uint32_t kSegBits = 1u << (kSegLog - 1);
constexpr uint32_t kSegWords = kSegBits / 32;
constexpr int kWave = 64;
constexpr uint64_t kGroupMax = 1ull << 50;   // K-prime products stay below 2^50 (mulmod bound)
constexpr uint32_t kKmodLdsGroups = 2048;     // K groups staged in LDS by the K mod p kernel (16 KB)
constexpr uint32_t kFusedGroupsMax = 512;     // primes dividing K for K mod p formed in the large branch
constexpr uint32_t kDSmall = 4096;            // d <= kDSmall: m -> row from a residue table of d entries

// Prime decades of the per-decade counters: decade i holds the primes 10^i <= p < 10^(i+1)
// (every p < 2^64 falls in one of them).
constexpr int kDecades = 20;
enum DecSlot { DC_PRIMES = 0, DC_RAW, DC_HITS, DC_SOLVES, DC_LEVELS, DC_COUNT };

// Counters in cs_diag order.
enum DiagSlot {
  D_NPRIMES = 0, D_SMALL_PRIMES, D_LARGE_PRIMES, D_SMALL_PAIRS, D_SMALL_MARKS,
  D_LARGE_RAW, D_LARGE_HITS, D_G_CALLS, D_G_LEVELS, D_ERROR, D_COUNT
};

// Error bits set by device-side checks.
enum ErrBits : uint32_t {
  E_ROWS = 1, E_COLS = 2, E_SOLVE = 4, E_TIERS = 8, E_PRIMES = 16
};

// Written by the device during preparation; read by later kernels of the same job.
struct JobCtrl {
  uint64_t n_lim;                    // primes <= limit
  uint64_t n_pP;                     // primes <= P
  uint64_t small_lo, small_dense, small_hi;   // prime indices of the small branch
  uint64_t small_single;             // first small prime above w (at most one mark per row)
  uint64_t tier_lo_idx;              // first prime index of tier 0
  uint64_t tier_idx[kMaxTiers];      // one past the last prime index of tier t
  uint64_t tier_item_base[kMaxTiers + 1];
  uint64_t n_items;
  uint32_t n_kgroups, n_kq, n_dq, error;
  uint32_t n_base, pad0;
  uint32_t dq[kMaxDq];
  uint64_t mq[kMaxDq];               // m_start mod dq[i]
  unsigned long long diag[D_COUNT];
  unsigned long long dec[DC_COUNT][kDecades];   // large-branch counters per prime decade
};

// Everything a kernel needs about one job.  Lives in device memory (written by a one-thread
// kernel that receives it as an argument, so no host-to-device copy is ever needed).
struct JobDev {
  uint64_t d, m_start, m_inc, limit, thr, p_lo, p_hi, n_m;
  uint32_t P, sl, w, n_x, row_words, large_mode;
  uint32_t tile_rows, n_windows, n_slices, hits_per_item;
  uint64_t small_unit_base;          // first small-branch unit of this job in a fused launch
  uint64_t dense_max;                // small primes <= dense_max are marked cooperatively
  uint64_t prime_cap;                // capacity of the prime table
  uint32_t n_tiers;
  uint32_t small_atomic;             // 1: the small branch merges its tiles with atomics (it runs
                                     // beside a large branch that ORs into the same bitmap)
  uint32_t d_small;                  // 1 if d <= kDSmall (rows from dpre, no per-m table lookups)
  uint32_t phi_d;                    // residues mod d coprime to d
  uint32_t r0_d;                     // m_start mod d
  uint32_t pre_r0;                   // coprime residues below r0_d
  double inv_d;                      // 1/d, correctly rounded
  uint32_t kmod_cached;              // 1: kmod already holds K mod p (a shared table); only mk is built
  uint32_t kmod_fused;               // 1: kmod and mk cover only the primes <= thr; the large branch
                                     // forms K mod p and m_start K mod p of its primes itself
  uint64_t wide_lo;                  // primes >= wide_lo take the exact 64-bit residue arithmetic
  // The large branch walks m of the residue classes mod m_step that can hold rows (bit c of
  // m_classes: m = c mod m_step coprime to it; m_step divides d), one class after the other:
  // 2 (odd m) when d is even, 6 (m = 1, 5 mod 6) with one solve per hit when 6 divides d, else 1.
  uint32_t m_step;
  uint32_t m_classes;
  uint32_t m0_mod_step;              // m_start mod m_step
  uint32_t branches;                 // branches this call runs (CS_BRANCH_*): what the prime counters count
  // Marks of the primes dividing d depend only on m mod d: one packed row (and its factor
  // count) per residue class coprime to d, built once per job and OR-ed into each row's tile.
  uint32_t dpat_on;                  // pattern table built for this job
  uint32_t dpat_apply;               // this call's prime range covers every prime dividing d
  uint32_t* dpat;                    // phi(d) x row_words words
  uint32_t* dpat_cnt;                // phi(d) counts
  const uint16_t* dres;              // the phi(d) residues coprime to d, ascending
  const uint16_t* dpre;              // d entries: bit 15 = coprime to d, bits 0-14 = coprime residues below
  uint64_t tier_lo;                  // tier 0 holds primes in (tier_lo, tier_hi[0]]
  uint64_t tier_hi[kMaxTiers];
  uint32_t tier_chunks[kMaxTiers];
  const uint64_t* primes;            // shared ascending prime table
  const uint64_t* n_primes;          // its length (device scalar)
  uint64_t* kmod;                    // K mod p per prime index (< n_lim)
  uint64_t* mk;                      // m_start*K mod p per prime index
  int32_t* row_of;                   // m - m_start -> row or -1
  uint32_t* m_off;                   // row -> m - m_start
  uint32_t* row_blk;                 // scan scratch for the row map
  uint2* coltab;                     // per 32 offsets j = X + sl: {column mask, columns before}
  uint64_t* kgroups;                 // products of the primes dividing K, each < 2^50
  uint32_t* kq;                      // primes dividing K (q <= P, q not dividing d)
  uint32_t* bitmap;
  uint32_t* counts;
  uint8_t* hitbytes;                 // one byte per (row, column slot) or null: large hits by store
  uint32_t fold_keep;                // 1: the fold leaves the byte counters as they are (no later call
                                     // of this preparation adds to them; the next one clears them)
  // List scatter: large hits appended as cells (row << cell_shift) | col into chunks of kListChunk cells
  // (one chunk open per wavefront), then grouped by buckets of bkt_rows rows and OR-ed / counted
  // into the outputs through LDS tiles.
  uint32_t* list_pool;               // list_chunks * kListChunk cells
  uint32_t* list_fill;               // per chunk: cells written
  unsigned long long* list_cursor;   // chunks handed out (beyond list_chunks: pool exhausted)
  uint32_t* list_sorted;             // cells grouped by bucket
  uint32_t* bkt_count;               // n_bkt + 1
  uint32_t* bkt_base;                // n_bkt + 1: exclusive prefix of bkt_count
  uint32_t* bkt_cursor;              // n_bkt + 1 bucket cursors
  uint32_t* list_super;              // per group of buckets: cells counted by the large branch, bases, cursors
                                     // (3 x (kListSupers + 1) words)
  uint64_t list_chunks;
  uint32_t n_bkt, bkt_rows;          // bkt_rows = 2^(bkt_shift - cell_shift)
  uint32_t bkt_per_super;            // 2^super_shift buckets per first-level group
  uint32_t cell_shift;               // cell = (row << cell_shift) | col, 2^cell_shift >= n_x
  uint32_t bkt_shift, super_shift;
  JobCtrl* ctrl;
};

constexpr uint32_t kListChunk = 4096;        // cells per list chunk
constexpr uint32_t kMaxBuckets = 8192;       // row buckets of the list scatter
constexpr uint32_t kListTileBytes = 60 * 1024;   // LDS tile of one bucket: rows x row_words words + counts
constexpr uint32_t kListChunksPerBlock = 256;    // chunks per block of the grouping kernels
constexpr uint32_t kListSupers = 64;             // first-level groups of buckets
constexpr uint32_t kListMaxPerSuper = kMaxBuckets / kListSupers;
constexpr uint32_t kListPiece = 1u << 18;        // cells per second-level block step
constexpr uint32_t kListPart2X = 32;             // second-level blocks per group

}  // namespace cs

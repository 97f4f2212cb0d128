// HIP kernels of the Combined Sieve for gfx950 (wave64, 256 CUs, fp64 at full VALU rate).
//
// Pipeline of one job (Sections 3.1-3.3 of the paper):
//   primes  segmented sieve of Eratosthenes in LDS, compacted to an ascending table
//   prep    primes dividing K grouped into products < 2^50; prime factors of d
//   kmod    K mod p (the cached residue of Eq. 1) and m_start*K mod p per prime
//   rows    m -> row map (gcd(m, d) = 1) and columns X -> column map (gcd(X, K) = 1)
//   small   primes p <= thr: every (row, p) residue, offsets marked in LDS row tiles
//   large   primes p >  thr: Eq. 3 solved by Eq. 5 (per hit, or for the first hit with
//           three-gap steps after it); hits scattered by atomics, byte counters or a cell list
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "arith.h"
#include "arith_wide.h"
#include "device.h"
#include "launch.h"

namespace cs {

// ------------------------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------------------------
// A device-memory pointer typed as global (address space 1).  Pointers read from a JobDev are
// generic, and accesses through them compile to flat instructions, which also count against the
// LDS wait counter: an LDS read behind a flat atomic then waits for the atomic to reach memory.
// Through a global pointer the same accesses are global instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> gbl(T* p) { return (gptr<T>)p; }

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// number of table entries <= x (table ascending)
__device__ uint64_t upper_index(const uint64_t* t, uint64_t n, uint64_t x) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (t[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Column of offset j = X + sl from the table {mask, columns before} per 32 offsets, or false
// if X is not a column (gcd(X, K) > 1).
// Column-table entry {mask, columns before} as one 64-bit word (mask in the low half).
__device__ __forceinline__ uint64_t ct_entry(const uint2* ct, uint32_t i) {
  return reinterpret_cast<const uint64_t*>(ct)[i];
}
__device__ __forceinline__ uint64_t ct_entry(gptr<const uint2> ct, uint32_t i) {
  return ((gptr<const uint64_t>)ct)[i];
}
template <class CT>
__device__ __forceinline__ bool lookup_col(CT ct, uint32_t jj, uint32_t* col) {
  const uint64_t e = ct_entry(ct, jj >> 5);
  const uint32_t mask = (uint32_t)e, before = (uint32_t)(e >> 32);
  const uint32_t b = jj & 31;
  if (!((mask >> b) & 1u)) return false;
  *col = before + __popc(mask & ((1u << b) - 1u));
  return true;
}

// Block-wide exclusive scan of one uint32 per thread (blockDim.x <= 1024, multiple of 64).
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) sh[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint32_t s = (lane < nw) ? sh[lane] : 0;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      uint32_t y = __shfl_up(s, o, kWave);
      if (lane >= o) s += y;
    }
    if (lane < nw) sh[lane] = s;           // inclusive per-wave totals
  }
  __syncthreads();
  uint32_t before = (wid > 0 ? sh[wid - 1] : 0) + x - v;
  if (total) *total = sh[nw - 1];
  __syncthreads();
  return before;
}

// ------------------------------------------------------------------------------------------
// small kernels
// ------------------------------------------------------------------------------------------
__global__ void k_write_job(JobDev jd, JobDev* dst) { *dst = jd; }

struct UploadChunk {
  uint8_t bytes[2048];
};
__global__ void k_upload(UploadChunk c, uint8_t* dst, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.bytes[i];
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t s = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += s) p[i] = v;
}

__global__ void k_zero_ctrl(JobCtrl* c) {
  uint32_t* w = reinterpret_cast<uint32_t*>(c);
  for (uint32_t i = threadIdx.x; i < sizeof(JobCtrl) / 4; i += blockDim.x) w[i] = 0;
}

// ------------------------------------------------------------------------------------------
// Prime table: segmented sieve of Eratosthenes, odd numbers only.
// Segment s covers [s*2^19, (s+1)*2^19); bit i stands for n = s*2^19 + 2i + 1.
// ------------------------------------------------------------------------------------------

// Odd base primes <= isqrt(lim) (lim < 2^42, so < 2^21), one workgroup, LDS bit sieve over
// windows of 2^20 integers: the first window finds its primes from its own bits, the second
// marks the multiples of the first window's primes up to its square root (< 1449).
__global__ __launch_bounds__(1024) void k_base_primes(uint64_t lim, uint32_t* base, uint32_t* n_base) {
  constexpr uint32_t kWin = 1u << 20;                       // integers per window
  constexpr uint32_t kWords = (kWin / 2) / 32;              // odd numbers of a window
  constexpr uint32_t kPer = kWords / 1024;                  // 16 words per thread
  __shared__ uint32_t bits[kWords];
  uint64_t root = (uint64_t)sqrt((double)lim);
  while (root * root > lim) --root;
  while ((root + 1) * (root + 1) <= lim) ++root;
  uint32_t total = 0;
  for (uint32_t win = 0; win < 2; ++win) {
    const uint64_t w_lo = (uint64_t)win * kWin;             // bit b stands for w_lo + 2b + 1
    if (w_lo > root) break;
    const uint64_t w_hi = min<uint64_t>(w_lo + kWin - 1, root);
    const uint32_t nb = (uint32_t)((w_hi - w_lo + 1) / 2);  // odd numbers in [w_lo, w_hi]
    const uint32_t nw = (nb + 31) / 32;
    for (uint32_t i = threadIdx.x; i < kWords; i += blockDim.x) bits[i] = 0;
    __syncthreads();
    if (win == 0) {
      for (uint32_t q = 3; (uint64_t)q * q <= w_hi; q += 2) {
        bool comp = (bits[(q >> 1) >> 5] >> ((q >> 1) & 31)) & 1;   // uniform read after barrier
        if (!comp) {
          for (uint64_t n = (uint64_t)q * q + 2ull * q * threadIdx.x; n <= w_hi; n += 2ull * q * blockDim.x) {
            uint32_t b = (uint32_t)(n >> 1);
            atomicOr(&bits[b >> 5], 1u << (b & 31));
          }
        }
        __syncthreads();
      }
    } else {
      // the first window's primes (already in base[], written before the last barrier)
      for (uint32_t i = 0; i < total; ++i) {
        const uint64_t q = base[i];
        if (q * q > w_hi) break;
        uint64_t st = ((w_lo + q - 1) / q) * q;
        if (st < q * q) st = q * q;
        if ((st & 1) == 0) st += q;                        // odd multiples only
        for (uint64_t n = st + 2ull * q * threadIdx.x; n <= w_hi; n += 2ull * q * blockDim.x) {
          const uint32_t b = (uint32_t)((n - w_lo) >> 1);
          atomicOr(&bits[b >> 5], 1u << (b & 31));
        }
      }
      __syncthreads();
    }
    // bit b unmarked with 3 <= w_lo + 2b + 1 <= root is an odd prime
    uint32_t mine[kPer];
    uint32_t c = 0;
#pragma unroll
    for (uint32_t t = 0; t < kPer; ++t) {
      const uint32_t u = threadIdx.x * kPer + t;
      uint32_t m = 0;
      if (u < nw) {
        m = ~bits[u];
        if (win == 0 && u == 0) m &= ~1u;                    // n = 1
        if (u == nw - 1 && (nb & 31)) m &= (1u << (nb & 31)) - 1;
      }
      mine[t] = m;
      c += __popc(m);
    }
    __syncthreads();                                         // bits[] is free from here on
    uint32_t tot;
    uint32_t off = total + block_exclusive_scan(c, bits, &tot);
#pragma unroll
    for (uint32_t t = 0; t < kPer; ++t) {
      uint32_t m = mine[t];
      const uint32_t u = threadIdx.x * kPer + t;
      while (m) {
        uint32_t b = __ffs(m) - 1;
        m &= m - 1;
        base[off++] = (uint32_t)(w_lo + 2 * (u * 32 + b) + 1);
      }
    }
    total += tot;
    __syncthreads();                                         // base[] written, bits[] reusable
  }
  if (threadIdx.x == 0) *n_base = total;
}

// One workgroup per segment: mark odd composites in LDS, write prime flags and the count.
// Bits 0, Q, 2Q, ... of a 32-bit word.
__host__ __device__ constexpr uint32_t every_qth(uint32_t Q) {
  uint32_t m = 0;
  for (uint32_t b = 0; b < 32; b += Q) m |= 1u << b;
  return m;
}

// Periodic marks of the odd multiples of a small prime Q (below 32, so every word holds one
// or more): bit b stands for n = lo + 2b + 1, and Q | n iff b = b0 (mod Q) with
// b0 = (Q - (lo + 1) mod Q) (Q + 1)/2 mod Q.  A thread fills words u0, u0 + kStride, ...; the
// marks of word u are bits ph, ph + Q, ... with ph = (b0 - 32u) mod Q, which moves by
// (32 kStride) mod Q from one of its words to the next.
template <uint32_t Q>
__device__ __forceinline__ uint32_t pat_phase(uint64_t lo, uint32_t u0) {
  const uint32_t b0 = (uint32_t)(((Q - (lo + 1) % Q) * ((Q + 1) / 2)) % Q);
  return (b0 + Q * 32u - (u0 % Q) * (32u % Q)) % Q;
}

template <uint32_t Q, uint32_t kStride>
__device__ __forceinline__ uint32_t pat_next(uint32_t& ph) {
  const uint32_t w = every_qth(Q) << ph;
  constexpr uint32_t D = (kStride * 32u) % Q;
  ph = ph >= D ? ph - D : ph + Q - D;
  return w;
}

// The first odd multiple of q at or above max(lo, q^2).  kWide: lo up to 2^64 (exact 64-bit
// remainder); otherwise lo < 2^42, where the fp64 quotient is exact.
template <bool kWide>
__device__ __forceinline__ uint64_t first_odd_multiple(uint64_t lo, uint64_t q) {
  uint64_t st;
  if constexpr (kWide) {
    const uint64_t r = mod64(lo, q, 1.0 / (double)q);
    st = r ? lo + (q - r) : lo;
  } else {
    st = (uint64_t)(ceil((double)lo / (double)q)) * q;
  }
  if (st < q * q) st = q * q;
  if ((st & 1) == 0) st += q;
  return st;
}

// Base primes per chunk of the segment sieve, and the prime below which whole waves mark one
// prime (a prime from there on has at most 2^18 / 1024 = 256 odd multiples in a segment and is
// marked by one thread).
constexpr uint32_t kSieveChunk = 512;
constexpr uint32_t kSieveWaveMax = 1024;
constexpr uint32_t kSieveThreads = 512;   // workgroup size of the segment sieve
// bits of 3, 5, ..., 31 themselves in word 0 of segment 0 (n = 2b + 1)
constexpr uint32_t kPatPrimeBits = (1u << 1) | (1u << 2) | (1u << 3) | (1u << 5) | (1u << 6) | (1u << 8) |
                                   (1u << 9) | (1u << 11) | (1u << 14) | (1u << 15);

// BT, NT: types of the base-prime table and of its length (uint32_t for the LDS-sieved base below
// 2^21; uint64_t for the level-2 table of limits from 2^42, which starts with the prime 2).
template <bool kWide, class BT, class NT>
__global__ __launch_bounds__(kSieveThreads) void k_sieve_segments(uint64_t lim, uint64_t seg0, uint64_t n_seg,
                                                        const BT* __restrict__ base,
                                                        const NT* __restrict__ n_base_p,
                                                        uint32_t* __restrict__ flags,
                                                        uint32_t* __restrict__ seg_count) {
  __shared__ uint32_t bits[kSegWords];
  __shared__ uint32_t cq[kSieveChunk];     // a chunk of base primes
  __shared__ uint32_t cb[kSieveChunk];     // the first bit each marks in the segment, ~0u for none
  __shared__ uint32_t sh[32];
  const uint64_t n_base = *n_base_p;
  uint64_t i_first = 0;                    // the first base prime above 31
  while (i_first < n_base && base[i_first] <= 31) ++i_first;
  for (uint64_t s = blockIdx.x; s < n_seg; s += gridDim.x) {
    const uint64_t gs = seg0 + s;                                  // segment of the whole range
    const uint64_t lo = gs << kSegLog;
    const uint64_t hi = min(lo + (1ull << kSegLog) - 1, lim);     // inclusive
    // The odd multiples of the primes 3 to 31 (over half of all marks, and the ones whose atomics
    // would collide most) come from periodic word patterns.  A multiple below q^2 is composite
    // too, so the patterns need no q^2 start; only the primes themselves (segment 0) are taken
    // back.
    {
      const uint32_t u0 = threadIdx.x;
      uint32_t p3 = pat_phase<3>(lo, u0), p5 = pat_phase<5>(lo, u0), p7 = pat_phase<7>(lo, u0);
      uint32_t p11 = pat_phase<11>(lo, u0), p13 = pat_phase<13>(lo, u0), p17 = pat_phase<17>(lo, u0);
      uint32_t p19 = pat_phase<19>(lo, u0), p23 = pat_phase<23>(lo, u0), p29 = pat_phase<29>(lo, u0);
      uint32_t p31 = pat_phase<31>(lo, u0);
      constexpr uint32_t T = kSieveThreads;
      for (uint32_t u = u0; u < kSegWords; u += T) {
        uint32_t w = pat_next<3, T>(p3) | pat_next<5, T>(p5) | pat_next<7, T>(p7) | pat_next<11, T>(p11) |
                     pat_next<13, T>(p13) | pat_next<17, T>(p17) | pat_next<19, T>(p19) | pat_next<23, T>(p23) |
                     pat_next<29, T>(p29) | pat_next<31, T>(p31);
        if (gs == 0 && u == 0) w &= ~kPatPrimeBits;
        bits[u] = w;
      }
    }
    const uint32_t nbits = (uint32_t)((hi - lo + 1) / 2);          // bits standing for n <= hi
    // The base primes above 13, a chunk at a time: first every thread finds the first marked bit
    // of its primes of the chunk (one division per prime and segment), then the primes below
    // kSieveWaveMax are marked by whole waves, one prime per wave at a time with lanes q apart,
    // and the larger ones (fewer marks each) one prime per thread.
    for (uint64_t c0 = i_first; c0 < n_base; c0 += kSieveChunk) {
      const uint64_t q_lead = base[c0];
      if (q_lead * q_lead > hi) break;                             // uniform: the primes are sorted
      const uint32_t nc = (uint32_t)min<uint64_t>(kSieveChunk, n_base - c0);
      __syncthreads();                                             // patterns / last chunk done
      for (uint32_t k = threadIdx.x; k < nc; k += blockDim.x) {
        const uint64_t q = base[c0 + k];
        uint32_t b0 = ~0u;
        if (q * q <= hi) {
          const uint64_t st = first_odd_multiple<kWide>(lo, q);
          if (st <= hi) b0 = (uint32_t)((st - lo) >> 1);
        }
        cq[k] = (uint32_t)q;
        cb[k] = b0;
      }
      __syncthreads();
      const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave, nwav = blockDim.x / kWave;
      for (uint32_t k = wid; k < nc; k += nwav) {
        const uint32_t q = cq[k];
        if (q >= kSieveWaveMax) break;
        const uint32_t b0 = cb[k];
        if (b0 == ~0u) continue;
        for (uint32_t b = b0 + lane * q; b < nbits; b += kWave * q) atomicOr(&bits[b >> 5], 1u << (b & 31));
      }
      for (uint32_t k = threadIdx.x; k < nc; k += blockDim.x) {
        const uint32_t q = cq[k];
        const uint32_t b0 = cb[k];
        if (q < kSieveWaveMax || b0 == ~0u) continue;
        if (q >= nbits) {                                          // one multiple (and b + q could wrap)
          atomicOr(&bits[b0 >> 5], 1u << (b0 & 31));
          continue;
        }
        for (uint32_t b = b0; b < nbits; b += q) atomicOr(&bits[b >> 5], 1u << (b & 31));
      }
    }
    __syncthreads();
    uint32_t c = 0;
    for (uint32_t u = threadIdx.x; u < kSegWords; u += blockDim.x) {
      uint32_t m = ~bits[u];
      if (gs == 0 && u == 0) m &= ~1u;                              // n = 1 is not prime
      const uint32_t first = u * 32;
      if (first >= nbits) m = 0;
      else if (nbits - first < 32) m &= (1u << (nbits - first)) - 1;
      flags[s * kSegWords + u] = m;
      c += __popc(m);
    }
    uint32_t tot;
    block_exclusive_scan(c, sh, &tot);
    if (threadIdx.x == 0) seg_count[s] = tot + ((gs == 0 && lim >= 2) ? 1u : 0u);  // the prime 2
    __syncthreads();
  }
}

// Exclusive scan of segment counts (one workgroup, loops over chunks).
__global__ __launch_bounds__(1024) void k_scan_counts(const uint32_t* __restrict__ cnt, uint64_t n,
                                                      uint64_t* __restrict__ off, uint64_t* total) {
  __shared__ uint32_t sh[32];
  uint64_t carry = 0;
  for (uint64_t b = 0; b < n; b += blockDim.x) {
    uint64_t i = b + threadIdx.x;
    uint32_t v = i < n ? cnt[i] : 0;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(v, sh, &tot);
    if (i < n) off[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

// Ordered compaction of the prime flags: 256 consecutive words per step, so reads are
// coalesced and each step's primes land in one contiguous run of the table.  Each wavefront
// scans its 64 words with cross-lane operations, gathers the bit positions of their primes in its
// own LDS region and writes them with consecutive lanes at consecutive addresses; the only
// workgroup barrier per step publishes the wavefronts' totals (double-buffered by step parity).
__global__ __launch_bounds__(256) void k_compact_primes(uint64_t seg0, uint64_t n_seg, const uint32_t* __restrict__ flags,
                                                        const uint64_t* __restrict__ off,
                                                        uint64_t* __restrict__ primes, uint64_t cap) {
  constexpr uint32_t kWaves = 256 / kWave;
  __shared__ uint32_t wtot[2][kWaves];
  __shared__ uint16_t pos_bits[kWaves][kWave * 32];   // a wavefront's primes: bit index in its words
  const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  uint32_t parity = 0;
  for (uint64_t s = blockIdx.x; s < n_seg; s += gridDim.x) {
    uint64_t base = off[s];
    if (seg0 + s == 0) {
      if (threadIdx.x == 0 && cap > 0) primes[0] = 2;
      base += 1;
    }
    const uint64_t lo = (seg0 + s) << kSegLog;
    constexpr uint32_t kAhead = 4;                               // steps whose words are loaded together
    static_assert((kSegWords / 256) % kAhead == 0, "whole batches of steps");
    for (uint32_t step0 = 0; step0 < kSegWords / 256; step0 += kAhead) {
      uint32_t mw[kAhead];
#pragma unroll
      for (uint32_t i = 0; i < kAhead; ++i) mw[i] = flags[s * kSegWords + (step0 + i) * 256 + threadIdx.x];
#pragma unroll
      for (uint32_t i = 0; i < kAhead; ++i, parity ^= 1) {
        const uint32_t step = step0 + i;
        uint32_t m = mw[i];
        const uint32_t c = __popc(m);
        uint32_t x = c;                                          // inclusive scan over the wavefront
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const uint32_t y = __shfl_up(x, o, kWave);
          if (lane >= (uint32_t)o) x += y;
        }
        const uint32_t wave_total = __shfl(x, kWave - 1, kWave);
        uint32_t k = x - c;
        while (m) {
          const uint32_t b = __ffs(m) - 1;
          m &= m - 1;
          pos_bits[wid][k++] = (uint16_t)(lane * 32 + b);
        }
        if (lane == 0) wtot[parity][wid] = wave_total;
        __syncthreads();
        uint64_t wbase = base;
        uint32_t step_total = 0;
#pragma unroll
        for (uint32_t w = 0; w < kWaves; ++w) {
          const uint32_t t = wtot[parity][w];
          if (w < wid) wbase += t;
          step_total += t;
        }
        const uint64_t wave_lo = lo + 2ull * (step * 256 + wid * kWave) * 32 + 1;
        for (uint32_t t = lane; t < wave_total; t += kWave) {
          const uint64_t g = wbase + t;
          if (g < cap) primes[g] = wave_lo + 2ull * pos_bits[wid][t];
        }
        base += step_total;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Job preparation
// ------------------------------------------------------------------------------------------

// One thread: primes dividing K grouped into products < 2^50, prime factors of d, and
// m_start mod each of them.
__global__ void k_prep_tables(JobDev* jobs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  JobDev& j = jobs[blockIdx.y];
  JobCtrl& c = *j.ctrl;
  uint64_t np = *j.n_primes;
  if (np > j.prime_cap) {
    atomicOr(&c.error, (uint32_t)E_PRIMES);
    np = j.prime_cap;
  }
  c.n_pP = upper_index(j.primes, np, j.P);
  c.n_lim = upper_index(j.primes, np, j.limit);
  uint64_t g = 1;
  uint32_t ng = 0, nkq = 0, ndq = 0;
  for (uint64_t i = 0; i < c.n_pP; ++i) {
    const uint64_t q = j.primes[i];
    if (j.d % q == 0) {
      if (ndq < kMaxDq) { c.dq[ndq] = (uint32_t)q; c.mq[ndq] = j.m_start % q; }
      ++ndq;
      continue;
    }
    j.kq[nkq++] = (uint32_t)q;
    if (g > (kGroupMax - 1) / q) { j.kgroups[ng++] = g; g = q; }
    else g *= q;
  }
  if (g > 1) j.kgroups[ng++] = g;
  c.n_kgroups = ng;
  c.n_kq = nkq;
  c.n_dq = ndq;
  c.diag[D_NPRIMES] = np;
}

// A later chunk of the prime range (the chunked sieve): the table now holds the primes of the
// chunk alone, so only its length and the primes it counts change; K's groups, the prime factors
// of d and the row and column tables stay those derived from the first chunk.
__global__ void k_chunk_bounds(JobDev* jobs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  JobDev& j = jobs[blockIdx.y];
  JobCtrl& c = *j.ctrl;
  uint64_t np = *j.n_primes;
  if (np > j.prime_cap) {
    atomicOr(&c.error, (uint32_t)E_PRIMES);
    np = j.prime_cap;
  }
  c.n_lim = upper_index(j.primes, np, j.limit);
  c.diag[D_NPRIMES] += c.n_lim;
}

// Prefix of the per-job prime counts (primes <= limit) over the jobs of a launch.
__global__ void k_lim_scan(const JobDev* jobs, uint32_t n_jobs, uint64_t* base) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t s = 0;
  for (uint32_t i = 0; i < n_jobs; ++i) {
    base[i] = s;
    const JobDev& j = jobs[i];
    const uint64_t n = j.ctrl->n_lim;
    s += j.kmod_fused ? upper_index(j.primes, n, j.thr) : n;   // fused: the small branch's primes only
  }
  base[n_jobs] = s;
}

// K mod p and m_start*K mod p for every prime index < n_lim of every job (Eq. 1's cached
// residue); the index space of all jobs is flattened so one launch covers a whole batch.
__device__ __forceinline__ const JobDev& job_of_index(const JobDev* __restrict__ jobs, uint32_t n_jobs,
                                                      const uint64_t* __restrict__ lim_base, uint64_t g,
                                                      uint64_t* i) {
  uint32_t lo = 0, hi = n_jobs;                     // job: last base <= g
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (lim_base[mid] <= g) lo = mid; else hi = mid;
  }
  *i = g - lim_base[lo];
  return jobs[lo];
}

// K mod p and m_start*K mod p of one prime p >= 2^20 (odd) with the exact 64-bit arithmetic.
__device__ __noinline__ void kmod_wide_one(const JobDev& j, uint64_t i, uint64_t p) {
  const Mont64 m = mont_setup(p);
  uint64_t k;
  if (j.kmod_cached) {
    k = gbl(j.kmod)[i];
  } else {
    k = kmod64(m, gbl(j.kgroups), gbl(j.ctrl)->n_kgroups);
    gbl(j.kmod)[i] = k;
  }
  gbl(j.mk)[i] = mulmod_m(m, umod64(j.m_start, p), k);
}

// K mod p and m_start*K mod p for every prime index < n_lim of every job (Eq. 1's cached
// residue); the index space of all jobs is flattened so one launch covers a whole batch.  Each
// thread takes two indices and interleaves their multiplication chains.
__global__ __launch_bounds__(256) void k_kmod(const JobDev* __restrict__ jobs, uint32_t n_jobs,
                                              const uint64_t* __restrict__ lim_base) {
  // a single job's K groups as doubles in LDS: the product chain below then reads no memory
  __shared__ double s_g[kKmodLdsGroups];
  const uint32_t ng_lds = n_jobs == 1 && !jobs[0].kmod_cached ? gbl(jobs[0].ctrl)->n_kgroups : 0u;
  const bool g_lds = ng_lds > 0 && ng_lds <= kKmodLdsGroups;
  if (g_lds) {
    for (uint32_t i = threadIdx.x; i < ng_lds; i += blockDim.x) s_g[i] = (double)gbl(jobs[0].kgroups)[i];
    __syncthreads();
  }
  const uint64_t total = lim_base[n_jobs];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t g0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g0 < total; g0 += 2 * stride) {
    const uint64_t g1 = g0 + stride;
    uint64_t i0, i1 = 0;
    const JobDev& j0 = job_of_index(jobs, n_jobs, lim_base, g0, &i0);
    const bool two = g1 < total;
    const JobDev& j1 = two ? job_of_index(jobs, n_jobs, lim_base, g1, &i1) : j0;
    if (!two) i1 = i0;
    const uint64_t p0 = gbl(j0.primes)[i0], p1 = gbl(j1.primes)[i1];
    if (p0 >= j0.wide_lo || p1 >= j1.wide_lo) {
      // 64-bit primes: Montgomery products of K's groups (the rare top of a wide range)
      kmod_wide_one(j0, i0, p0);
      if (two) kmod_wide_one(j1, i1, p1);
      continue;
    }
    const double v0 = 1.0 / (double)p0, v1 = 1.0 / (double)p1;
    uint64_t r0, r1;
    if (&j0 == &j1 && !j0.kmod_cached) {
      // Eq. 1: the product of K's prime groups (each below 2^50) mod p, all in fp64
      const uint32_t ng = gbl(j0.ctrl)->n_kgroups;
      const gptr<const uint64_t> G = gbl(j0.kgroups);
      const double pd0 = (double)p0, pd1 = (double)p1;
      // lazily reduced products (|x| < 2.32p all along), one full reduction at the end
      double x0 = p0 == 1 ? 0.0 : 1.0, x1 = p1 == 1 ? 0.0 : 1.0;
      if (g_lds) {
        for (uint32_t t = 0; t < ng; ++t) {
          const double gg = s_g[t];
          x0 = mulmod_f64_lazy(x0, gg, pd0, v0);
          x1 = mulmod_f64_lazy(x1, gg, pd1, v1);
        }
      } else {
        for (uint32_t t = 0; t < ng; ++t) {
          const double gg = (double)G[t];
          x0 = mulmod_f64_lazy(x0, gg, pd0, v0);
          x1 = mulmod_f64_lazy(x1, gg, pd1, v1);
        }
      }
      r0 = (uint64_t)reduce_f64(x0, pd0, v0);
      r1 = (uint64_t)reduce_f64(x1, pd1, v1);
    } else {
      auto kof = [](const JobDev& j, uint64_t i, uint64_t p, double v) {
        if (j.kmod_cached) return (uint64_t)gbl(j.kmod)[i];
        uint64_t r = 1 % p;
        for (uint32_t t = 0; t < gbl(j.ctrl)->n_kgroups; ++t) r = mulmod(r, gbl(j.kgroups)[t], p, v);
        return r;
      };
      r0 = kof(j0, i0, p0, v0);
      r1 = kof(j1, i1, p1, v1);
    }
    // m_start K mod p: both factors below p < 2^42, so the fp64 product applies
    if (!j0.kmod_cached) gbl(j0.kmod)[i0] = r0;
    gbl(j0.mk)[i0] = (uint64_t)mulmod_f64((double)mod64(j0.m_start, p0, v0), (double)r0, (double)p0, v0);
    if (two) {
      if (!j1.kmod_cached) gbl(j1.kmod)[i1] = r1;
      gbl(j1.mk)[i1] = (uint64_t)mulmod_f64((double)mod64(j1.m_start, p1, v1), (double)r1, (double)p1, v1);
    }
  }
}

// Clears the outputs of every job (blockIdx.y = job).
__global__ void k_fill_jobs(const JobDev* __restrict__ jobs) {
  const JobDev& j = jobs[blockIdx.y];
  const uint64_t nb = j.n_m * (uint64_t)j.row_words;
  const uint64_t s = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nb; i += s) j.bitmap[i] = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < j.n_m; i += s) j.counts[i] = 0;
}

// Clears the control block of every job (blockIdx.y = job).
__global__ void k_zero_ctrls(const JobDev* __restrict__ jobs) {
  uint32_t* w = reinterpret_cast<uint32_t*>(jobs[blockIdx.y].ctrl);
  for (uint32_t i = threadIdx.x; i < sizeof(JobCtrl) / 4; i += blockDim.x) w[i] = 0;
}

// Stand-alone K mod p for the cs_kmod entry point.
__global__ __launch_bounds__(256) void k_kmod_list(const uint64_t* __restrict__ primes, uint64_t n,
                                                   const uint64_t* __restrict__ G, uint32_t ng,
                                                   uint64_t* __restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t p = primes[i];
    if (p >= (1ull << 42)) {                       // exact 64-bit products for the widest primes
      out[i] = kmod64(mont_setup(p), G, ng);
      continue;
    }
    const double pinv = 1.0 / (double)p;
    uint64_t r = 1 % p;
    for (uint32_t g = 0; g < ng; ++g) r = mulmod(r, G[g], p, pinv);
    out[i] = r;
  }
}

__device__ __forceinline__ bool m_coprime(const JobCtrl& c, uint64_t o) {
  const uint32_t nd = c.n_dq < kMaxDq ? c.n_dq : kMaxDq;
  for (uint32_t t = 0; t < nd; ++t)
    if ((c.mq[t] + o) % c.dq[t] == 0) return false;
  return true;
}

constexpr uint32_t kRowBlock = 1024;

__global__ __launch_bounds__(256) void k_rows_count(const JobDev* __restrict__ jobs) {
  __shared__ uint32_t sh[32];
  const JobDev& j = jobs[blockIdx.y];
  const uint64_t nb = (j.m_inc + kRowBlock - 1) / kRowBlock;
  for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    uint32_t c = 0;
    for (uint32_t t = threadIdx.x; t < kRowBlock; t += blockDim.x) {
      uint64_t o = b * kRowBlock + t;
      if (o < j.m_inc && m_coprime(*j.ctrl, o)) ++c;
    }
    uint32_t tot;
    block_exclusive_scan(c, sh, &tot);
    if (threadIdx.x == 0) j.row_blk[b] = tot;
  }
}

__global__ __launch_bounds__(1024) void k_rows_scan(const JobDev* __restrict__ jobs) {
  __shared__ uint32_t sh[32];
  const JobDev& j = jobs[blockIdx.y];
  const uint64_t nb = (j.m_inc + kRowBlock - 1) / kRowBlock;
  uint64_t carry = 0;
  for (uint64_t b = 0; b < nb; b += blockDim.x) {
    uint64_t i = b + threadIdx.x;
    uint32_t v = i < nb ? j.row_blk[i] : 0;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(v, sh, &tot);
    if (i < nb) j.row_blk[i] = (uint32_t)(carry + ex);
    carry += tot;
  }
  if (threadIdx.x == 0 && carry != j.n_m) atomicOr(&j.ctrl->error, (uint32_t)E_ROWS);
}

__global__ __launch_bounds__(1024) void k_rows_write(const JobDev* __restrict__ jobs) {
  __shared__ uint32_t sh[32];
  const JobDev& j = jobs[blockIdx.y];
  const uint64_t nb = (j.m_inc + kRowBlock - 1) / kRowBlock;
  for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const uint64_t o = b * kRowBlock + threadIdx.x;
    const bool ok = o < j.m_inc && m_coprime(*j.ctrl, o);
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(ok ? 1u : 0u, sh, &tot);
    const uint32_t row = j.row_blk[b] + ex;
    if (o < j.m_inc) j.row_of[o] = ok ? (int32_t)row : -1;
    if (ok && row < j.n_m) j.m_off[row] = (uint32_t)o;
  }
}

// Column table: j = X + sl in [0, 2 sl]; X is a column iff gcd(X, K) = 1.
__global__ __launch_bounds__(256) void k_cols_mask(const JobDev* __restrict__ jobs) {
  const JobDev& j = jobs[blockIdx.y];
  const uint32_t S = 2 * j.sl + 1;
  const uint32_t nkq = j.ctrl->n_kq;
  const uint32_t nwords = (S + 31) / 32;
  for (uint32_t base = blockIdx.x * blockDim.x; base < nwords * 32; base += gridDim.x * blockDim.x) {
    const uint32_t jj = base + threadIdx.x;
    bool col = false;
    if (jj < S) {
      const int64_t X = (int64_t)jj - (int64_t)j.sl;
      const uint64_t ax = (uint64_t)(X < 0 ? -X : X);
      if (ax == 0) {
        col = (nkq == 0);                       // gcd(0, K) = K
      } else {
        col = true;
        for (uint32_t t = 0; t < nkq; ++t) {
          const uint32_t q = j.kq[t];
          if (q > ax) break;
          if (ax % q == 0) { col = false; break; }
        }
      }
    }
    const uint64_t bal = __ballot(col);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    if (lane == 0 || lane == 32) {
      const uint32_t word = jj / 32;
      if (word < nwords) j.coltab[word].x = (uint32_t)(bal >> lane);
    }
  }
}

__global__ __launch_bounds__(1024) void k_cols_prefix(const JobDev* __restrict__ jobs) {
  __shared__ uint32_t sh[32];
  const JobDev& j = jobs[blockIdx.y];
  const uint32_t nwords = (2 * j.sl + 1 + 31) / 32;
  uint32_t carry = 0;
  for (uint32_t b = 0; b < nwords; b += blockDim.x) {
    const uint32_t i = b + threadIdx.x;
    const uint32_t v = i < nwords ? __popc(j.coltab[i].x) : 0;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, sh, &tot);
    if (i < nwords) j.coltab[i].y = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && carry != j.n_x) atomicOr(&j.ctrl->error, (uint32_t)E_COLS);
}

// Prime-index bounds of the branches and the large-branch work items of one job.
__global__ void k_prep_bounds(JobDev* jobs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  JobDev& j = jobs[blockIdx.y];
  JobCtrl& c = *j.ctrl;
  const uint64_t n = c.n_lim;
  const uint64_t* pr = j.primes;
  const uint64_t lo = j.p_lo > 2 ? j.p_lo : 2;
  const uint64_t hi = j.p_hi < j.limit ? j.p_hi : j.limit;
  const uint64_t small_hi_v = hi < j.thr ? hi : j.thr;
  c.small_lo = upper_index(pr, n, lo - 1);
  c.small_hi = (small_hi_v >= lo) ? upper_index(pr, n, small_hi_v) : c.small_lo;
  uint64_t dm = j.dense_max < small_hi_v ? j.dense_max : small_hi_v;
  c.small_dense = (dm >= lo) ? upper_index(pr, n, dm) : c.small_lo;
  if (c.small_dense > c.small_hi) c.small_dense = c.small_hi;
  if (c.small_dense < c.small_lo) c.small_dense = c.small_lo;
  c.small_single = upper_index(pr, n, j.w);
  if (c.small_single > c.small_hi) c.small_single = c.small_hi;
  if (c.small_single < c.small_dense) c.small_single = c.small_dense;
  c.tier_lo_idx = upper_index(pr, n, j.tier_lo);
  uint64_t prev = c.tier_lo_idx, items = 0;
  for (uint32_t t = 0; t < j.n_tiers; ++t) {
    uint64_t e = upper_index(pr, n, j.tier_hi[t]);
    if (e < prev) e = prev;
    c.tier_idx[t] = e;
    c.tier_item_base[t] = items;
    items += (e - prev) * (uint64_t)j.tier_chunks[t];
    prev = e;
  }
  c.tier_item_base[j.n_tiers] = items;
  c.n_items = items;
  // each call counts the primes of the branches it runs (CS_BRANCH_ALL = 0, SMALL = 1, LARGE = 2)
  if (j.branches != 2u) c.diag[D_SMALL_PRIMES] += c.small_hi - c.small_lo;
  if (j.branches != 1u) c.diag[D_LARGE_PRIMES] += prev - c.tier_lo_idx;
}

// Prefix of large-branch item counts over the jobs of a launch.
__global__ void k_items_scan(const JobDev* jobs, uint32_t n_jobs, uint64_t* base) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t s = 0;
  for (uint32_t i = 0; i < n_jobs; ++i) {
    base[i] = s;
    s += jobs[i].ctrl->n_items;
  }
  base[n_jobs] = s;
}

// Per residue class c of m mod d (c coprime to d): the packed column marks and factor count
// of the primes q dividing d.  For those primes N mod q = (m mod q)(K mod q) mod q depends
// only on m mod d, so one row per class replaces their per-row marking (Eq. 1).
__global__ __launch_bounds__(256) void k_dpattern(const JobDev* __restrict__ jobs) {
  extern __shared__ uint32_t row[];
  __shared__ uint32_t kmq[kMaxDq];
  __shared__ uint32_t cnt_sh;
  const JobDev& j = jobs[blockIdx.y];
  if (!j.dpat_on) return;
  const JobCtrl& c = *j.ctrl;
  const uint32_t nd = c.n_dq < kMaxDq ? c.n_dq : kMaxDq;
  if (threadIdx.x < nd) {
    const uint32_t q = c.dq[threadIdx.x];
    uint32_t r = 1 % q;
    for (uint32_t i = 0; i < c.n_kq; ++i) r = (uint32_t)(((uint64_t)r * (j.kq[i] % q)) % q);
    kmq[threadIdx.x] = r;                           // K mod q
  }
  __syncthreads();
  const uint32_t rw = j.row_words, w = j.w;
  for (uint32_t cls = blockIdx.x; cls < j.phi_d; cls += gridDim.x) {
    for (uint32_t u = threadIdx.x; u < rw; u += blockDim.x) row[u] = 0;
    if (threadIdx.x == 0) cnt_sh = 0;
    __syncthreads();
    const uint32_t res = j.dres[cls];
    uint32_t cc = 0;
    for (uint32_t t = 0; t < nd; ++t) {
      const uint32_t q = c.dq[t];
      const uint32_t nq = (uint32_t)(((uint64_t)(res % q) * kmq[t]) % q);     // N mod q
      const uint32_t s0 = (j.sl % q + q - nq) % q;                            // j = X + sl
      for (uint64_t jj = s0 + (uint64_t)threadIdx.x * q; jj <= w; jj += (uint64_t)blockDim.x * q) {
        uint32_t col;
        if (lookup_col(j.coltab, (uint32_t)jj, &col)) {
          atomicOr(&row[col >> 5], 1u << (col & 31));
          ++cc;
        }
      }
    }
    cc = wave_sum_u32(cc);
    if ((threadIdx.x & (kWave - 1)) == 0 && cc) atomicAdd(&cnt_sh, cc);
    __syncthreads();
    for (uint32_t u = threadIdx.x; u < rw; u += blockDim.x) j.dpat[(uint64_t)cls * rw + u] = row[u];
    if (threadIdx.x == 0) j.dpat_cnt[cls] = cnt_sh;
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------
// Small-prime branch (Section 3.1 space-time tradeoff; Section 5: p/S < C_mult).
// One unit = (job, window of tile_rows consecutive rows, prime slice).  For every row and
// prime, N mod p = m*K mod p comes from the cached K mod p (Eq. 1), and the offsets
// X = -N (mod p) of the window are marked in an LDS tile of packed column bits.
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t p) {
  return a >= b ? a - b : a + p - b;
}

// Marks of the small primes [s_lo, s_hi) in one tile (rows row_lo.. of the job), into the LDS tile
// and row counts.  Inlined once with the column table in LDS and once in global memory so that
// each copy reads it through its own address space.
struct SmallArgs {
  const JobDev& j;
  uint64_t small_dense, small_single;
  uint32_t* tile;
  uint32_t* cnt;
  const uint32_t* moff;
  uint32_t R, rw, w;
  uint64_t s_lo, s_hi;
  bool dpat;
  uint32_t lane, wid, nwaves;
};

// Small primes above w (at most one mark per row), residues below 2^31: prime indices
// [i_lo, i_hi), one lane per prime.  Between rows the offset s (the X + sl with p | m K + X)
// steps by -dm k (mod p) for the row gap dm, which is the same for every lane: the multiples
// g k mod p for g < 16 sit in registers and the gap indexes them (a scalar index), and a gap of
// 16 or more takes one modular product.
// Where a wave's primes hit few of the tile's rows (p >= R (w + 1) / 2: at most about two hits
// per lane), a first pass only steps the offsets and keeps the rows with s <= w as bits; a second
// pass visits each lane's own hit rows (the offset again from the first row's by one modular
// product), looks the column up and marks it, with the row count added by an LDS atomic.  Below
// that bound the column lookup runs for every lane and row without a branch, two rows at a time
// so that their LDS reads overlap, and row r's marks by the wave accumulate in lane r of one
// register (rows <= 64), added to the tile's row counts once at the end.
template <bool kHit, class CT>
__device__ __forceinline__ void small_single_marks(const SmallArgs& a, CT ct, uint64_t i_lo, uint64_t i_hi,
                                                   unsigned long long& n_pairs, unsigned long long& n_marks) {
  const JobDev& j = a.j;
  uint32_t* tile = a.tile;
  const uint32_t R = a.R, rw = a.rw, w = a.w, lane = a.lane;
  const bool dpat = a.dpat;
  const uint64_t sl = j.sl;
  const uint32_t P = j.P;
  const gptr<const uint64_t> primes = gbl(j.primes);
  const gptr<const uint64_t> kmod = gbl(j.kmod);
  const gptr<const uint64_t> mkp = gbl(j.mk);
  const uint32_t moffv = lane < R ? a.moff[lane] : 0u;         // lane r: m offset of row r
  // the hit-row pass steps a fixed kHitRows rows, those past R repeating the last row (gap 0),
  // when every row gap of the tile indexes the register table
  constexpr uint32_t kHitRows = 16;
  const uint32_t moffc = R ? a.moff[lane < R ? lane : R - 1] : 0u;
  const uint32_t gapv = lane + 1 < R ? a.moff[lane + 1] - a.moff[lane] : 0u;
  const bool hit_rows_ok = R >= 1 && R <= kHitRows && __ballot(gapv >= 16u) == 0;
  uint32_t cntv = 0;                                           // lane r: this wave's marks in row r
  uint32_t nmv = 0;                                            // this lane's marks by hit rows
  for (uint64_t ib = i_lo; ib < i_hi; ib += blockDim.x) {
    const uint64_t i = ib + threadIdx.x;
    bool act = i < i_hi;
    uint64_t p = 3, k = 0, mk = 0;
    if (act) { p = primes[i]; k = kmod[i]; mk = mkp[i]; }
    act = act && k != 0 && !(dpat && p <= P);
    const double pinv = 1.0 / (double)p;
    const uint32_t p32 = (uint32_t)p;
    uint32_t km[16];                                           // g k mod p
    km[0] = 0;
#pragma unroll
    for (int g = 1; g < 16; ++g) {
      const uint32_t t = km[g - 1] + (uint32_t)k;              // < 2p < 2^32
      km[g] = t >= p32 ? t - p32 : t;
    }
    uint32_t s0;
    {
      const uint32_t o0 = __builtin_amdgcn_readfirstlane(moffv);
      uint64_t rn = mk + mulmod(o0, k, p, pinv);
      rn = rn >= p ? rn - p : rn;
      s0 = (uint32_t)sub_mod(sl, rn, p);                        // sl < w < p
    }
    auto advance = [&](uint32_t s, uint32_t dm) -> uint32_t {
      const uint32_t kd = dm < 16u ? km[dm] : (uint32_t)mulmod(dm, k, p, pinv);
      const uint32_t t = s - kd;
      return s >= kd ? t : t + p32;
    };
    const uint32_t na = (uint32_t)__popcll(__ballot(act));
    if (lane == 0) n_pairs += (unsigned long long)na * R;
    // the wave's smallest prime sits in its first lane (an idle first lane: an idle wave)
    const uint32_t p_first = __builtin_amdgcn_readfirstlane(p32);
    if (kHit && hit_rows_ok && (uint64_t)R * (w + 1ull) <= 2ull * p_first) {
      const uint32_t o0 = __builtin_amdgcn_readfirstlane(moffc);
      uint32_t hitm = s0 <= w ? 1u : 0u;                       // bit r: row r has s <= w
      uint32_t sr = s0, o_prev = o0;
#pragma unroll
      for (uint32_t r = 1; r < kHitRows; ++r) {
        const uint32_t o = __builtin_amdgcn_readlane(moffc, r);
        const uint32_t kd = km[o - o_prev];                    // a scalar index below 16
        o_prev = o;
        const uint32_t t = sr - kd;
        sr = min(t, t + p32);                                  // t wrapped above 2^31 when sr < kd
        hitm |= sr <= w ? 1u << r : 0u;
      }
      hitm &= (1u << R) - 1u;                                  // R <= 16
      if (!act) hitm = 0;
      while (hitm) {
        const uint32_t r = (uint32_t)__builtin_ctz(hitm);
        hitm &= hitm - 1;
        const uint32_t kd = (uint32_t)mulmod(a.moff[r] - o0, k, p, pinv);
        const uint32_t sh = s0 >= kd ? s0 - kd : s0 + p32 - kd;
        const uint64_t e = ct_entry(ct, sh >> 5);
        const uint32_t b = sh & 31u;
        if (((uint32_t)e >> b) & 1u) {
          const uint32_t col = (uint32_t)(e >> 32) + __popc((uint32_t)e & ((1u << b) - 1u));
          atomicOr(&tile[r * rw + (col >> 5)], 1u << (col & 31));
          atomicAdd(&a.cnt[r], 1u);
          ++nmv;
        }
      }
      continue;
    }
    for (uint32_t r = 0; r < R; r += 2) {
      const bool two = r + 1 < R;                              // the same for every lane
      const uint32_t o_r = __builtin_amdgcn_readlane(moffv, r);
      const uint32_t o_r1 = two ? __builtin_amdgcn_readlane(moffv, r + 1) : o_r;
      const uint32_t s1 = two ? advance(s0, o_r1 - o_r) : s0;
      const bool h0 = act && s0 <= w;
      const bool h1 = two && act && s1 <= w;
      const uint32_t j0 = h0 ? s0 : 0u, j1 = h1 ? s1 : 0u;
      const uint64_t e0 = ct_entry(ct, j0 >> 5);
      const uint64_t e1 = ct_entry(ct, j1 >> 5);
      const uint32_t b0 = j0 & 31u, b1 = j1 & 31u;
      const bool ok0 = h0 && (((uint32_t)e0 >> b0) & 1u);
      const bool ok1 = h1 && (((uint32_t)e1 >> b1) & 1u);
      if (ok0) {
        const uint32_t col = (uint32_t)(e0 >> 32) + __popc((uint32_t)e0 & ((1u << b0) - 1u));
        atomicOr(&tile[r * rw + (col >> 5)], 1u << (col & 31));
      }
      if (ok1) {
        const uint32_t col = (uint32_t)(e1 >> 32) + __popc((uint32_t)e1 & ((1u << b1) - 1u));
        atomicOr(&tile[(r + 1) * rw + (col >> 5)], 1u << (col & 31));
      }
      const uint32_t t0 = (uint32_t)__popcll(__ballot(ok0));
      const uint32_t t1 = (uint32_t)__popcll(__ballot(ok1));
      cntv += lane == r ? t0 : (lane == r + 1 ? t1 : 0u);
      if (r + 2 < R) {
        const uint32_t o_r2 = __builtin_amdgcn_readlane(moffv, r + 2);
        s0 = advance(s1, o_r2 - o_r1);
      }
    }
  }
  if (lane < R && cntv) atomicAdd(&a.cnt[lane], cntv);
  const uint32_t tot = wave_sum_u32(cntv + nmv);
  if (lane == 0) n_marks += tot;
}

template <bool kHit>
__device__ __forceinline__ void small_marks(const SmallArgs& a, const uint2* __restrict__ ct,
                                            unsigned long long& n_pairs, unsigned long long& n_marks) {
  const JobDev& j = a.j;
  uint32_t* tile = a.tile;
  uint32_t* cnt = a.cnt;
  const uint32_t R = a.R, rw = a.rw, w = a.w, lane = a.lane, wid = a.wid, nwaves = a.nwaves;
  const uint64_t s_lo = a.s_lo, s_hi = a.s_hi;
  const bool dpat = a.dpat;
  const uint64_t sl = j.sl;
  const uint32_t P = j.P;
  const gptr<const uint64_t> primes = gbl(j.primes);
  const gptr<const uint64_t> kmod = gbl(j.kmod);
  const gptr<const uint64_t> mkp = gbl(j.mk);
  // dense primes: one wave per prime, lanes stride over its multiples in each row
  const uint64_t d_hi = min(s_hi, max(a.small_dense, s_lo));
  for (uint64_t i = s_lo + wid; i < d_hi; i += nwaves) {
    const uint64_t p = primes[i];
    const uint64_t k = kmod[i];
    if (k == 0) continue;                         // p | K: never divides a column's N + X
    if (dpat && p <= P) continue;               // p | d: marked by the class pattern
    const double pinv = 1.0 / (double)p;
    const uint64_t mk = mkp[i];
    const uint64_t slp = mod64(sl, p, pinv);
    for (uint32_t r = 0; r < R; ++r) {
      const uint32_t o = a.moff[r];
      uint64_t rn = mk + mulmod(o, k, p, pinv);
      rn = rn >= p ? rn - p : rn;                 // N mod p
      const uint64_t s0 = sub_mod(slp, rn, p);    // first offset j = X + sl with p | N + X
      uint32_t cc = 0;
      for (uint64_t jj = s0 + (uint64_t)lane * p; jj <= w; jj += (uint64_t)kWave * p) {
        uint32_t col;
        if (lookup_col(ct, (uint32_t)jj, &col)) {
          atomicOr(&tile[r * rw + (col >> 5)], 1u << (col & 31));
          ++cc;
        }
      }
      cc = wave_sum_u32(cc);
      if (lane == 0) {
        if (cc) atomicAdd(&cnt[r], cc);
        n_pairs += 1;
        n_marks += cc;
      }
    }
  }
  // sparse primes: one lane per prime, rows in order, residues stepped by the m gaps
  const uint64_t sp_lo = max(s_lo, min(a.small_dense, s_hi));
  if (j.thr < (1ull << 31)) {
    // primes above w: at most one mark per row
    const uint64_t sg_lo = max(sp_lo, min(a.small_single, s_hi));
    if (R <= kWave && sg_lo < s_hi) small_single_marks<kHit>(a, ct, sg_lo, s_hi, n_pairs, n_marks);
    const uint64_t sp_hi = R <= kWave ? sg_lo : s_hi;
    // the others: every small prime (<= thr) is below 2^31, so residues sit in 32-bit registers
    // (s + p - k < 2^32, jj + p < 2^32), and the marks of a row are counted by ballots (a lane
    // marks a row at most once when p > w; the full reduction runs only for a row where some
    // lane marked twice)
    for (uint64_t ib = sp_lo; ib < sp_hi; ib += blockDim.x) {
      const uint64_t i = ib + threadIdx.x;
      bool act = i < sp_hi;
      uint64_t p = 3, k = 0, mk = 0;
      if (act) { p = primes[i]; k = kmod[i]; mk = mkp[i]; }
      act = act && k != 0 && !(dpat && p <= P);
      const double pinv = 1.0 / (double)p;
      const uint32_t p32 = (uint32_t)p, k32 = (uint32_t)k;
      uint32_t s32 = 0;
      uint32_t o_prev = 0;
      if (R > 0) {
        o_prev = a.moff[0];
        uint64_t rn = mk + mulmod(o_prev, k, p, pinv);
        rn = rn >= p ? rn - p : rn;
        s32 = (uint32_t)sub_mod(mod64(sl, p, pinv), rn, p);
      }
      const uint32_t na = (uint32_t)__popcll(__ballot(act));
      for (uint32_t r = 0; r < R; ++r) {
        if (r > 0) {
          const uint32_t o = a.moff[r];
          const uint32_t dm = o - o_prev;           // same for every lane
          o_prev = o;
          if (dm <= 12) {
            for (uint32_t t = 0; t < dm; ++t) s32 = s32 >= k32 ? s32 - k32 : s32 + p32 - k32;
          } else {
            s32 = (uint32_t)sub_mod(s32, mulmod(dm, k, p, pinv), p);
          }
        }
        uint32_t cc = 0;
        if (act) {
          for (uint32_t jj = s32; jj <= w; jj += p32) {
            uint32_t col;
            if (lookup_col(ct, jj, &col)) {
              atomicOr(&tile[r * rw + (col >> 5)], 1u << (col & 31));
              ++cc;
            }
          }
        }
        const unsigned long long many = __ballot(cc > 1);
        const uint32_t tot = many ? wave_sum_u32(cc) : (uint32_t)__popcll(__ballot(cc != 0));
        if (lane == 0) {
          if (tot) atomicAdd(&cnt[r], tot);
          n_marks += tot;
        }
      }
      if (lane == 0) n_pairs += (unsigned long long)na * R;
    }
    return;
  }
  for (uint64_t ib = sp_lo; ib < s_hi; ib += blockDim.x) {
    const uint64_t i = ib + threadIdx.x;
    bool act = i < s_hi;
    uint64_t p = 3, k = 0, mk = 0;
    if (act) { p = primes[i]; k = kmod[i]; mk = mkp[i]; }
    act = act && k != 0 && !(dpat && p <= P);
    const double pinv = 1.0 / (double)p;
    uint64_t s = 0;
    uint32_t o_prev = 0;
    if (R > 0) {
      o_prev = a.moff[0];
      uint64_t rn = mk + mulmod(o_prev, k, p, pinv);
      rn = rn >= p ? rn - p : rn;
      s = sub_mod(mod64(sl, p, pinv), rn, p);
    }
    for (uint32_t r = 0; r < R; ++r) {
      if (r > 0) {
        const uint32_t o = a.moff[r];
        const uint32_t dm = o - o_prev;           // same for every lane
        o_prev = o;
        if (dm <= 12) {
          for (uint32_t t = 0; t < dm; ++t) s = sub_mod(s, k, p);
        } else {
          s = sub_mod(s, mulmod(dm, k, p, pinv), p);
        }
      }
      uint32_t cc = 0;
      if (act) {
        for (uint64_t jj = s; jj <= w; jj += p) {
          uint32_t col;
          if (lookup_col(ct, (uint32_t)jj, &col)) {
            atomicOr(&tile[r * rw + (col >> 5)], 1u << (col & 31));
            ++cc;
          }
        }
      }
      const uint32_t na = (uint32_t)__popcll(__ballot(act));
      cc = wave_sum_u32(cc);
      if (lane == 0) {
        if (cc) atomicAdd(&cnt[r], cc);
        n_pairs += na;
        n_marks += cc;
      }
    }
  }
}

// One small-branch unit (a window of tile_rows rows and a slice of the small primes) of job j,
// by the whole workgroup: unit `local` of the job.  lds: [column table, lds_ct_words uint2][tile
// rows x row_words][counts][m offsets]; ct_ready: the job's column table is already in place.
template <bool kHit>
__device__ __forceinline__ void small_unit(const JobDev& j, uint64_t local, uint32_t* lds, uint32_t lds_ct_words,
                                           bool ct_ready, unsigned long long& n_pairs, unsigned long long& n_marks) {
  const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const uint32_t nwaves = blockDim.x / kWave;
  const auto& c = *gbl(j.ctrl);
  const uint64_t window = local / j.n_slices;
  const uint32_t slice = (uint32_t)(local % j.n_slices);
  const uint64_t row_lo = window * j.tile_rows;
  const uint64_t row_hi = min(row_lo + j.tile_rows, j.n_m);
  const uint32_t R = (uint32_t)(row_hi - row_lo);
  const uint32_t rw = j.row_words;
  const uint32_t w = j.w;
  // prime slice
  const uint64_t span = c.small_hi - c.small_lo;
  const uint64_t s_lo = c.small_lo + span * slice / j.n_slices;
  const uint64_t s_hi = c.small_lo + span * (slice + 1) / j.n_slices;
  // LDS: [column table][tile R x rw][counts R]
  const uint32_t nct = (2 * j.sl + 1 + 31) / 32;
  const bool ct_in_lds = nct <= lds_ct_words;
  uint2* ct_l = reinterpret_cast<uint2*>(lds);
  uint32_t* tile = lds + 2 * lds_ct_words;
  uint32_t* cnt = tile + (uint32_t)j.tile_rows * rw;
  uint32_t* moff = cnt + j.tile_rows;            // m - m_start of the tile's rows
  if (ct_in_lds && !ct_ready)
    for (uint32_t i = threadIdx.x; i < nct; i += blockDim.x) ct_l[i] = ((const uint2*)gbl(j.coltab))[i];
  for (uint32_t i = threadIdx.x; i < R * rw; i += blockDim.x) tile[i] = 0;
  for (uint32_t i = threadIdx.x; i < R; i += blockDim.x) {
    cnt[i] = 0;
    moff[i] = gbl(j.m_off)[row_lo + i];
  }
  __syncthreads();
  const bool dpat = j.dpat_apply != 0;
  if (dpat && slice == 0) {
    // primes dividing d: the row of this m's residue class (tile rows start cleared)
    const double dd = (double)j.d;
    for (uint32_t r = 0; r < R; ++r) {
      const double x = (double)j.r0_d + (double)moff[r];
      double rr = fma(-floor(x * j.inv_d), dd, x);
      rr = rr < 0.0 ? rr + dd : (rr >= dd ? rr - dd : rr);
      const uint32_t cls = gbl(j.dpre)[(uint32_t)rr] & 0x7fffu;
      const gptr<const uint32_t> src = gbl(j.dpat) + (uint64_t)cls * rw;
      for (uint32_t u = threadIdx.x; u < rw; u += blockDim.x) tile[r * rw + u] = src[u];
      if (threadIdx.x == 0) {
        const uint32_t pc = gbl(j.dpat_cnt)[cls];
        cnt[r] = pc;
        n_marks += pc;
      }
    }
    __syncthreads();
  }

  {
    SmallArgs a{j, c.small_dense, c.small_single, tile, cnt, moff, R, rw, w, s_lo, s_hi, dpat, lane, wid, nwaves};
    if (ct_in_lds) small_marks<kHit>(a, ct_l, n_pairs, n_marks);   // LDS column table
    else small_marks<kHit>(a, (const uint2*)gbl(j.coltab), n_pairs, n_marks);   // global column table
  }
  __syncthreads();
  // write the tile: rows of this unit belong to it alone unless the primes are sliced
  for (uint32_t r = 0; r < R; ++r) {
    const gptr<uint32_t> dst = gbl(j.bitmap) + (row_lo + r) * (uint64_t)rw;
    for (uint32_t u = threadIdx.x; u < rw; u += blockDim.x) {
      const uint32_t v = tile[r * rw + u];
      if (!v) continue;
      if (j.n_slices == 1 && !j.small_atomic) dst[u] |= v;
      else atomicOr((uint32_t*)(dst + u), v);
    }
  }
  for (uint32_t r = threadIdx.x; r < R; r += blockDim.x) {
    const uint32_t v = cnt[r];
    if (!v) continue;
    if (j.n_slices == 1 && !j.small_atomic) gbl(j.counts)[row_lo + r] += v;
    else atomicAdd((uint32_t*)(gbl(j.counts) + row_lo + r), v);
  }
  __syncthreads();
}

// kHit: the hit-row pass for the primes far above w (its own instance, so that the other keeps
// its register budget: jobs of few rows per prime range ran slower with the pass compiled in)
template <bool kHit>
__global__ __launch_bounds__(256) void k_small(const JobDev* __restrict__ jobs, uint32_t n_jobs,
                                               uint64_t total_units, uint32_t lds_ct_words) {
  extern __shared__ uint32_t lds[];
  const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const uint32_t nwaves = blockDim.x / kWave;
  unsigned long long n_pairs = 0, n_marks = 0;
  uint32_t ji = 0;                                   // units only grow: resume the job search
  for (uint64_t unit = blockIdx.x; unit < total_units; unit += gridDim.x) {
    while (ji + 1 < n_jobs && jobs[ji + 1].small_unit_base <= unit) ++ji;
    small_unit<kHit>(jobs[ji], unit - jobs[ji].small_unit_base, lds, lds_ct_words, false, n_pairs, n_marks);
  }
  // counters: one atomic per workgroup and counter (lane 0 of each wavefront holds its sums)
  __shared__ unsigned long long s_cnt[2][256 / kWave];
  if (lane == 0) {
    s_cnt[0][wid] = n_pairs;
    s_cnt[1][wid] = n_marks;
  }
  __syncthreads();
  if (threadIdx.x < 2 && n_jobs > 0) {
    unsigned long long v = 0;
    for (uint32_t i = 0; i < nwaves; ++i) v += s_cnt[threadIdx.x][i];
    if (v) atomicAdd((unsigned long long*)(gbl(jobs[0].ctrl->diag) + (threadIdx.x == 0 ? D_SMALL_PAIRS : D_SMALL_MARKS)), v);
  }
}

// ------------------------------------------------------------------------------------------
// Large-prime branch (Section 3.2-3.3).  One item = (job, prime, chunk of the m range).
// From the residue r of m*K + SL the next m with r <= 2*SL (Eq. 3, shifted form) comes from
// G of Eq. 5; each such m marks X = SL - r when gcd(m, d) = 1 and X is a column.
// ------------------------------------------------------------------------------------------
// Position of m = m_start + o relative to d: m_start mod d + o = dq * d + rd.  With the residue
// table of d this gives gcd(m, d) = 1 and the row of m with no per-m memory lookup.
struct MPos {
  uint32_t rd;
  uint32_t dq;
};

__device__ __forceinline__ void mpos_divmod(uint64_t x, uint32_t d, double inv_d, uint32_t* q, uint32_t* r) {
  const double xd = (double)x, dd = (double)d;
  double qq = floor(xd * inv_d);
  double rr = fma(-qq, dd, xd);
  if (rr < 0.0) { rr += dd; qq -= 1.0; }
  if (rr >= dd) { rr -= dd; qq += 1.0; }
  *q = (uint32_t)qq;
  *r = (uint32_t)rr;
}

// The same for a double holding an integer below 2^52.
__device__ __forceinline__ void mpos_divmod_d(double xd, uint32_t d, double inv_d, uint32_t* q, uint32_t* r) {
  const double dd = (double)d;
  double qq = floor(xd * inv_d);
  double rr = fma(-qq, dd, xd);
  if (rr < 0.0) { rr += dd; qq -= 1.0; }
  if (rr >= dd) { rr -= dd; qq += 1.0; }
  *q = (uint32_t)qq;
  *r = (uint32_t)rr;
}

__device__ __forceinline__ void mpos_add(MPos& s, uint32_t tq, uint32_t tr, uint32_t d) {
  s.rd += tr;
  s.dq += tq;
  if (s.rd >= d) { s.rd -= d; s.dq += 1; }
}

// Decade of p: i with 10^i <= p < 10^(i+1) (integer compares: exact for every p < 2^64).
__device__ __forceinline__ uint32_t decade_of(uint64_t p) {
  uint32_t dc = 0;
  uint64_t t = 10;
#pragma unroll
  for (int i = 1; i < kDecades; ++i) {
    dc += p >= t ? 1u : 0u;
    t *= 10;
  }
  return dc;
}

// Table accessors: LDS copies for a single-job launch, global memory otherwise.
template <bool kLds>
struct LargeTables {
  const uint2* ct;
  const uint16_t* dp;
  const double* kg;              // K's prime groups as doubles (K mod p formed in the kernel)
};
template <>
struct LargeTables<false> {
  gptr<const uint2> ct;
  gptr<const uint16_t> dp;
  gptr<const uint64_t> kg;
};

// Large-hit scatter variants (template argument kSc): 0 = atomic OR into the bitmap and atomic add
// into the row's count; 1 = one atomic add into a byte counter per (row, column), folded into the
// bitmap and the counts after the launch; 2 = append the cell row * n_x + col to this wavefront's
// chunk of the list pool (no atomic per hit), grouped and applied after the launch.
constexpr uint32_t kNoChunk = 0xffffffffu;
constexpr uint32_t kPoolFull = 0xfffffffeu;

// floor(a / b) for a, b < 2^52 through the fp64 quotient and one exact correction each way
// (a 64-bit integer division is a long emulated sequence on the GPU).
__device__ __forceinline__ uint64_t div_small(uint64_t a, uint64_t b) {
  const double bd = (double)b;
  double q = floor((double)a / bd);
  const double r = fma(-q, bd, (double)a);
  q += (r < 0.0) ? -1.0 : ((r >= bd) ? 1.0 : 0.0);
  return (uint64_t)q;
}

// What the hit path needs of a job, copied into registers once per item: the kernel's own stores
// (bitmap, counts, list cells) could alias a JobDev in global memory as far as the compiler knows,
// so reading these through the JobDev inside the walking loop reloads them at every step.
struct HitCtx {
  gptr<const int32_t> row_of;
  gptr<uint32_t> bitmap;
  gptr<uint32_t> counts;
  gptr<uint8_t> hitbytes;
  gptr<uint32_t> list_pool;
  gptr<uint32_t> list_fill;
  gptr<unsigned long long> list_cursor;
  uint64_t list_chunks;
  uint32_t d_small, phi_d, pre_r0, row_words, cell_shift, sup_shift;
};

__device__ __forceinline__ HitCtx hit_ctx(const JobDev& j) {
  HitCtx h;
  h.row_of = gbl(j.row_of);
  h.bitmap = gbl(j.bitmap);
  h.counts = gbl(j.counts);
  h.hitbytes = gbl(j.hitbytes);
  h.list_pool = gbl(j.list_pool);
  h.list_fill = gbl(j.list_fill);
  h.list_cursor = gbl(j.list_cursor);
  h.list_chunks = j.list_chunks;
  h.d_small = j.d_small;
  h.phi_d = j.phi_d;
  h.pre_r0 = j.pre_r0;
  h.row_words = j.row_words;
  h.cell_shift = j.cell_shift;
  h.sup_shift = j.bkt_shift + j.super_shift;
  return h;
}

// The open list chunk of a wavefront and the cells written to it.  Kept in registers, identical
// in every lane that takes part in a step; lanes that left the walking loop early catch up at the
// end of the item (list_sync).
struct ListReg {
  uint32_t chunk, fill;
};

// One append step, taken by every lane of the walking loop (ok = this lane has a hit): one ballot,
// consecutive slots in the open chunk, one 4-byte store per hit (one contiguous run per
// wavefront).  A full chunk is closed (its fill recorded) and a new one taken from the pool
// cursor; when the pool is exhausted, hits take the atomic path instead.
__device__ __forceinline__ void list_step(const HitCtx& j, ListReg& lr, bool ok,
                                          uint32_t cell, uint64_t row, uint32_t col, uint32_t* sup) {
  const unsigned long long act = __ballot(ok);
  if (act == 0) return;
  const uint32_t lane = __lane_id();
  const uint32_t n = (uint32_t)__popcll(act);
  const uint32_t rank = (uint32_t)__popcll(act & ((1ull << lane) - 1ull));
  const uint32_t leader = (uint32_t)__ffsll((long long)act) - 1u;
  // the state is the same in every participating lane: scalar copies make the tests below
  // uniform branches
  uint32_t chunk = __builtin_amdgcn_readfirstlane(lr.chunk);
  uint32_t fill = __builtin_amdgcn_readfirstlane(lr.fill);
  if (chunk == kNoChunk || (chunk != kPoolFull && fill + n > kListChunk)) {
    uint32_t nc = kPoolFull;
    if (lane == leader) {
      if (chunk != kNoChunk) j.list_fill[chunk] = fill;
      const unsigned long long c = atomicAdd((unsigned long long*)j.list_cursor, 1ull);
      if (c < j.list_chunks) nc = (uint32_t)c;
    }
    chunk = __builtin_amdgcn_readlane(nc, leader);
    fill = 0;
  }
  if (ok) {
    if (chunk != kPoolFull) {
      j.list_pool[(uint64_t)chunk * kListChunk + fill + rank] = cell;
      atomicAdd(&sup[cell >> j.sup_shift], 1u);     // the workgroup's cells per group of buckets
    } else {
      atomicOr((uint32_t*)(j.bitmap + row * j.row_words + (col >> 5)), 1u << (col & 31));
      atomicAdd((uint32_t*)(j.counts + row), 1u);
    }
  }
  lr.chunk = chunk;
  lr.fill = fill + n;
}

// Brings every lane that ran this item to the wavefront's latest list state: chunk ids grow with
// each allocation and fills grow within a chunk, so the latest state has the largest key
// (chunk + 1) << 32 | fill (kNoChunk maps to 0, kPoolFull to the top).  lkey: this wavefront's
// LDS slot, only ever raised.
__device__ __forceinline__ void list_sync(ListReg& lr, unsigned long long* lkey) {
  const unsigned long long key = ((unsigned long long)(uint32_t)(lr.chunk + 1u) << 32) | lr.fill;
  atomicMax(lkey, key);
  const unsigned long long k = *reinterpret_cast<volatile unsigned long long*>(lkey);
  lr.chunk = (uint32_t)(k >> 32) - 1u;
  lr.fill = (uint32_t)k;
}

template <bool kLds, int kSc>
__device__ __forceinline__ void record_hit(const HitCtx& j, const LargeTables<kLds>& T, uint64_t o, MPos mp,
                                           uint32_t jj, unsigned long long& useful, ListReg& lr, uint32_t* sup) {
  if constexpr (kSc == 2) {
    // every lane of the loop takes the step, with or without a hit
    bool ok;
    uint32_t row;
    if (j.d_small) {
      const uint32_t e = T.dp[mp.rd];
      ok = (e >> 15) != 0;                          // m shares a factor with d (Section 3.2)
      row = j.phi_d * mp.dq + (e & 0x7fffu) - j.pre_r0;
    } else {
      const int32_t r = j.row_of[o];
      ok = r >= 0;
      row = ok ? (uint32_t)r : 0u;
    }
    uint32_t col = 0;
    if (ok) ok = lookup_col(T.ct, jj, &col);        // X shares a factor with K
    list_step(j, lr, ok, ok ? ((row << j.cell_shift) | col) : 0u, row, col, sup);
    if (ok) ++useful;
    return;
  }
  // Both table reads are issued before either test, and the two tests (m coprime to d,
  // Section 3.2; X coprime to K) are one condition: one LDS round trip and one branch per step.
  const uint64_t ce = ct_entry(T.ct, jj >> 5);
  uint32_t row;                                     // rows < m_inc < 2^32
  bool ok;
  if (j.d_small) {
    const uint32_t e = T.dp[mp.rd];
    ok = (e >> 15) != 0;
    row = j.phi_d * mp.dq + (e & 0x7fffu) - j.pre_r0;
  } else {
    const int32_t r = j.row_of[o];
    ok = r >= 0;
    row = (uint32_t)r;
  }
  const uint32_t mask = (uint32_t)ce, b = jj & 31;
  ok = ok && ((mask >> b) & 1u);
  if (!ok) return;
  const uint32_t col = (uint32_t)(ce >> 32) + __popc(mask & ((1u << b) - 1u));
  if constexpr (kSc == 1) {
    gptr<uint32_t> cell = (gptr<uint32_t>)(j.hitbytes + (uint64_t)row * (j.row_words * 32u) + (col & ~3u));
    atomicAdd((uint32_t*)cell, 1u << (8 * (col & 3u)));
  } else {
    atomicOr((uint32_t*)(j.bitmap + (uint64_t)row * j.row_words + (col >> 5)), 1u << (col & 31));
    atomicAdd((uint32_t*)(j.counts + row), 1u);
  }
  ++useful;
}

// ------------------------------------------------------------------------------------------
// Large-prime branch (Section 3.2-3.3).  One item = (job, prime, chunk of the m range).
// From the residue r of m*K + SL the next m with r <= 2*SL (Eq. 3, shifted form) comes from
// G of Eq. 5; each such m marks X = SL - r when gcd(m, d) = 1 and X is a column.
// When d is even only odd m can be rows: the walk takes m = m0 + 2u (m0 the first odd m), whose
// residues step by 2K mod p, so Eq. 5 and the three-gap return times are those of 2K mod p and
// the even m are never visited.
// ------------------------------------------------------------------------------------------
// Per-lane counters of the large branch, for the decade of the lane's current prime (a lane's
// items only grow, so its primes change decade rarely); flushed into the workgroup's per-decade
// LDS counters when the decade changes and at the end.
struct LaneCount {
  unsigned long long raw, useful, calls, levels, n_pr;
  uint32_t cur_dec, err;
};

__device__ __forceinline__ void lane_count_init(LaneCount& lc) {
  lc.raw = lc.useful = lc.calls = lc.levels = lc.n_pr = 0;
  lc.cur_dec = kDecades;
  lc.err = 0;
}

__device__ __forceinline__ void flush_dec(LaneCount& lc, unsigned long long (*s_dec)[kDecades]) {
  const uint32_t d = lc.cur_dec;
  if (d < (uint32_t)kDecades) {
    if (lc.n_pr) atomicAdd(&s_dec[DC_PRIMES][d], lc.n_pr);
    if (lc.raw) atomicAdd(&s_dec[DC_RAW][d], lc.raw);
    if (lc.useful) atomicAdd(&s_dec[DC_HITS][d], lc.useful);
    if (lc.calls) atomicAdd(&s_dec[DC_SOLVES][d], lc.calls);
    if (lc.levels) atomicAdd(&s_dec[DC_LEVELS][d], lc.levels);
  }
  lc.raw = lc.useful = lc.calls = lc.levels = lc.n_pr = 0;
}

// One large-branch work item (prime, chunk of the m range) of job j: item `local` of the job's
// tiered item space.  t_last: the lane's tier of its previous item of this job (items only grow).
// kWide: the prime is at least 2^42 and its residues take the exact 64-bit arithmetic.
template <bool kLds, int kSc, bool kG, bool kWide = false>
__device__ __forceinline__ void large_item(const JobDev& j, const LargeTables<kLds>& T, uint64_t local,
                                           uint32_t& t_last, LaneCount& lc, unsigned long long (*s_dec)[kDecades],
                                           ListReg& lreg, unsigned long long* lkey, uint32_t* s_sup) {
  const auto& c = *gbl(j.ctrl);
  uint32_t t = t_last;
  while (t + 1 < j.n_tiers && c.tier_item_base[t + 1] <= local) ++t;
  t_last = t;
  const uint64_t li = local - c.tier_item_base[t];
  const uint32_t C = j.tier_chunks[t];
  // Item order.  One solve per hit: prime-major, so neighbouring lanes share (p, K mod p)
  // and walk the same sequence of moduli in Eq. 5's descent (less divergence).  Three-gap
  // stepping: chunk-major, so lanes running at the same time share an m-chunk and their
  // scattered marks stay within 1/C of the bitmap rows.
  const uint64_t t0 = (t == 0 ? c.tier_lo_idx : c.tier_idx[t - 1]);
  uint64_t chunk, pi;
  if (C == 1) {
    chunk = 0;
    pi = t0 + li;
  } else if (kG) {
    const uint64_t q = div_small(li, C);
    pi = t0 + q;
    chunk = li - q * C;
  } else {
    const uint64_t npt = c.tier_idx[t] - t0;
    chunk = div_small(li, npt);
    pi = t0 + (li - chunk * npt);
  }
  // the walk's positions: for each class c of m mod s (s = m_step), m = m_start + o_c + s u with
  // o_c = (c - m_start) mod s and u in [0, U); a chunk is a range of u, shared by the classes
  const uint32_t s = j.m_step;
  const uint64_t U = (j.m_inc + s - 1) / s;
  const uint64_t L = C == 1 ? U : div_small(U + C - 1, C);
  const uint64_t u_lo = (uint64_t)chunk * L;
  const uint64_t u_hi = min(u_lo + L, U);
  if (u_lo >= u_hi) return;

  const uint64_t p = gbl(j.primes)[pi];
  // K mod p (Eq. 1) and m_start K mod p: from the tables, or formed here as the product of K's
  // prime groups (each below 2^50) modulo p, lazily reduced, in fp64 with 1/p correctly rounded
  uint64_t k1, mk;
  if (!kWide && j.kmod_fused) {
    const double pd = (double)p, pcr = 1.0 / pd;
    const uint32_t ng = gbl(j.ctrl)->n_kgroups;
    // two interleaved chains (even and odd groups), joined by one more product
    double x0 = 1.0, x1 = 1.0;
    uint32_t t = 0;
    for (; t + 2 <= ng; t += 2) {
      x0 = mulmod_f64_lazy(x0, (double)T.kg[t], pd, pcr);
      x1 = mulmod_f64_lazy(x1, (double)T.kg[t + 1], pd, pcr);
    }
    if (t < ng) x0 = mulmod_f64_lazy(x0, (double)T.kg[t], pd, pcr);
    k1 = (uint64_t)reduce_f64(mulmod_f64_lazy(x0, reduce_f64(x1, pd, pcr), pd, pcr), pd, pcr);
    mk = (uint64_t)mulmod_f64((double)mod64(j.m_start, p, pcr), (double)k1, pd, pcr);
  } else {
    k1 = gbl(j.kmod)[pi];
    mk = gbl(j.mk)[pi];
  }
  {
    const uint32_t dc = decade_of(p);
    if (dc != lc.cur_dec) {
      flush_dec(lc, s_dec);
      lc.cur_dec = dc;
    }
    if (chunk == 0) ++lc.n_pr;                        // each prime once (chunk 0 always has positions)
  }
  uint64_t k;                                      // residue step of one walk position: s K mod p
  if constexpr (kWide) {
    k = k1;
    for (uint32_t i = 1; i < s; ++i) k = addmod64(k, k1, p);
  } else {
    k = s * k1;
    k -= k >= 4 * p ? 4 * p : 0;                   // s <= 6: s K mod p < 8p before these
    k -= k >= 2 * p ? 2 * p : 0;
    k -= k >= p ? p : 0;
  }
  const double pinv = recip((double)p);             // within an ulp: every quotient below is corrected
  Mont64 mt = {0, 0, 0};
  if constexpr (kWide) mt = mont_setup(p);
  const uint64_t w = j.w;
  const uint32_t d32 = (uint32_t)j.d;
  const double inv_d = j.inv_d;
  const bool d_small = j.d_small != 0;
  const HitCtx hc = hit_ctx(j);
  // k^-1 mod p (and, for three-gap stepping, the two return times) from one Euclid pass
  uint64_t kinv = 0;
  gaps3 g = {0, 0, 0, 0};
  if constexpr (kWide) {
    if (kG) {
      kinv = modinv64(k, p);
    } else if (!three_gap_euclid64(p, k, w, &g, &kinv)) {
      lc.err |= E_SOLVE;
      return;
    }
  } else {
    if (kG) {
      kinv = modinv(k, p);
    } else if (!three_gap_euclid(p, k, w, &g, &kinv, nullptr)) {
      lc.err |= E_SOLVE;
      return;
    }
  }
  // three-gap return times in offsets of m (a time past the chunk ends the walk, so the
  // quotients below only matter for the times that are taken); with 64-bit primes they are
  // capped at 2^33, beyond any range of m, so that they stay exact in fp64 and never overflow
  constexpr uint64_t kCap = 1ull << 33;
  const uint64_t sta = kWide ? (g.ta >= kCap / s ? kCap : s * g.ta) : s * g.ta;
  const uint64_t stb = kWide ? (g.tb >= kCap / s ? kCap : s * g.tb) : s * g.tb;
  const uint64_t tab = kWide ? min(sta + stb, kCap) : sta + stb;
  uint32_t aq = 0, ar = 0, bq = 0, br = 0, abq = 0, abr = 0;
  if (!kG && d_small) {
    mpos_divmod(sta, d32, inv_d, &aq, &ar);
    mpos_divmod(stb, d32, inv_d, &bq, &br);
    mpos_divmod(tab, d32, inv_d, &abq, &abr);
  }
  GCache gc;
  if constexpr (kG && !kWide) g_cache_build((double)p, (double)k, (double)w, &gc);
  for (uint32_t cls = 0; cls < s; ++cls) {
    // list scatter: lanes that left the previous class's walk early catch up on the wavefront's
    // chunk state before the next walk appends (every lane reaches this point)
    if constexpr (kSc == 2) {
      if (cls > 0) list_sync(lreg, lkey);
    }
    const uint64_t o_par = (cls + s - j.m0_mod_step) % s;
    const uint64_t o_lo = o_par + s * u_lo;
    // a class that cannot hold rows, or that ends before this chunk, is skipped
    if (!((j.m_classes >> cls) & 1u) || o_lo >= j.m_inc) continue;
    const uint64_t o_hi = min(o_par + s * u_hi, j.m_inc);   // visited o = o_par + s u < o_hi
    // residue of m*K + SL at m = m_start + o_lo
    uint64_t r;
    if constexpr (kWide) {
      r = addmod64(mk, mulmod_m(mt, o_lo, k1), p);      // o_lo < 2^32 < p
    } else {
      r = mk + mulmod(o_lo, k1, p, pinv);
      r = r >= p ? r - p : r;
    }
    r += j.sl;                                     // sl < w < thr < p
    r = r >= p ? r - p : r;
    uint64_t o = o_lo;
    MPos mp = {0, 0};
    if (d_small) mpos_divmod(j.r0_d + o_lo, d32, inv_d, &mp.dq, &mp.rd);

    if (kG && !kWide) {
      // one solve of Eq. 3 per hit; every value an integer below 2^45 held as a double, and the
      // first levels of Eq. 5's descent for (p, k) taken from the item's cache
      const double pd = (double)p, kd = (double)k, kinvd = (double)kinv, wd = (double)w, sd = (double)s;
      const double ohd = (double)o_hi;
      double rd = (double)r, od = (double)o;
      while (true) {
        if (rd > wd) {
          int lv = 0;
          double rn = 0.0;
          const double t = next_hit_cached(gc, kinvd, pinv, rd, wd, &rn, &lv);
          ++lc.calls;
          lc.levels += (unsigned)lv;
          if (t == 0.0) { lc.err |= E_SOLVE; break; }
          od = fma(sd, t, od);
          if (od >= ohd) break;
          rd = rn;
          if (d_small) {
            uint32_t tq, tr;
            mpos_divmod_d(sd * t, d32, inv_d, &tq, &tr);
            mpos_add(mp, tq, tr, d32);
          }
        }
        ++lc.raw;
        record_hit<kLds, kSc>(hc, T, (uint64_t)(uint32_t)od, mp, (uint32_t)(wd - rd), lc.useful, lreg, s_sup);
        od += sd;
        if (od >= ohd) break;
        if (d_small) mpos_add(mp, 0, s, d32);      // s <= d: one correction suffices
        rd += kd;
        rd = rd >= pd ? rd - pd : rd;
      }
    } else if (kG) {
      // one solve of Eq. 3 per hit (64-bit primes)
      while (true) {
        if (r > w) {
          int lv = 0;
          uint64_t rn;
          uint64_t tstep;
          if constexpr (kWide) tstep = next_hit64(mt, k, kinv, r, w, &rn, &lv);
          else tstep = next_hit(p, k, kinv, pinv, r, w, &rn, &lv);
          ++lc.calls;
          lc.levels += (unsigned)lv;
          if (tstep == 0) { lc.err |= E_SOLVE; break; }
          if (kWide && tstep > (o_hi - o) / s) break;   // past the range (and no overflow below)
          o += s * tstep;
          if (o >= o_hi) break;
          r = rn;
          if (d_small) {
            uint32_t tq, tr;
            mpos_divmod(s * tstep, d32, inv_d, &tq, &tr);
            mpos_add(mp, tq, tr, d32);
          }
        }
        ++lc.raw;
        record_hit<kLds, kSc>(hc, T, o, mp, (uint32_t)(w - r), lc.useful, lreg, s_sup);
        if ((o += s) >= o_hi) break;
        if (d_small) mpos_add(mp, 0, s, d32);      // s <= d: one correction suffices
        r += k;
        r = r >= p ? r - p : r;
      }
    } else {
      // three-gap stepping: one solve for the first hit, then the return times
      if (r > w) {
        uint64_t rn;
        int lv = 0;
        uint64_t tstep;
        if constexpr (kWide) {
          tstep = next_hit64(mt, k, kinv, r, w, &rn, &lv);
        } else {
          double rnd = 0.0;
          tstep = (uint64_t)next_hit_d((double)p, (double)k, (double)kinv, pinv, (double)r, (double)w, &rnd, &lv);
          rn = (uint64_t)rnd;
        }
        ++lc.calls;
        lc.levels += (unsigned)lv;
        if (tstep == 0) { lc.err |= E_SOLVE; break; }
        if (kWide && tstep > (o_hi - o) / s) continue;  // the class's first hit lies past the range
        o += s * tstep;
        r = rn;
        if (d_small && o < o_hi) {
          uint32_t tq, tr;
          mpos_divmod(s * tstep, d32, inv_d, &tq, &tr);
          mpos_add(mp, tq, tr, d32);
        }
      }
      const bool a_first = g.ta < g.tb;
      // every residue from here on is a hit's, at most w < 2^18, and so are a and b: 32-bit
      // arithmetic, and the three cases by selects rather than branches
      const uint32_t w32 = (uint32_t)w, a32 = (uint32_t)g.a, b32 = (uint32_t)g.b;
      uint32_t r32 = (uint32_t)r;
      while (o < o_hi) {
        ++lc.raw;
        record_hit<kLds, kSc>(hc, T, o, mp, w32 - r32, lc.useful, lreg, s_sup);
        const bool fa = r32 + a32 <= w32, fb = r32 >= b32;
        const bool ua = fa && (a_first || !fb);
        const bool ub = !ua && fb;
        o += ua ? sta : (ub ? stb : tab);
        r32 = r32 + (ub ? 0u : a32) - (ua ? 0u : b32);
        mpos_add(mp, ua ? aq : (ub ? bq : abq), ua ? ar : (ub ? br : abr), d32);
      }
    }
  }
}

template <bool kLds, int kSc, bool kG, bool kWide>
__global__ __launch_bounds__(256) void k_large(const JobDev* __restrict__ jobs, uint32_t n_jobs,
                                               const uint64_t* __restrict__ job_item_base,
                                               unsigned long long* __restrict__ diag,
                                               unsigned long long* __restrict__ dec, uint32_t lds_ct_words,
                                               uint32_t dpre_n) {
  extern __shared__ uint32_t lds[];
  __shared__ unsigned long long s_list[256 / kWave];   // per wavefront: latest list state (see list_sync)
  __shared__ unsigned long long s_dec[DC_COUNT][kDecades];   // the workgroup's counters per prime decade
  __shared__ uint32_t s_sup[kListSupers];                    // list scatter: cells per group of buckets
  const uint64_t total = job_item_base[n_jobs];
  if ((uint64_t)blockIdx.x * blockDim.x >= total) return;   // workgroups past the last item (uniform)
  // Issue priority over the small branch's waves that share the CUs: this kernel's rate is its
  // hit atomics in flight, and a busy small branch beside it otherwise takes the issue cycles
  // that keep them in flight (the small branch fills the cycles this kernel leaves).
  __builtin_amdgcn_s_setprio(1);
  unsigned long long* lkey = s_list + threadIdx.x / kWave;
  if (threadIdx.x < 256 / kWave) s_list[threadIdx.x] = 0ull;
  for (uint32_t i = threadIdx.x; i < DC_COUNT * kDecades; i += blockDim.x) (&s_dec[0][0])[i] = 0ull;
  if (threadIdx.x < kListSupers) s_sup[threadIdx.x] = 0u;
  __syncthreads();
  LargeTables<kLds> T;
  if constexpr (kLds) {
    const JobDev& j0 = jobs[0];
    uint2* ctl = reinterpret_cast<uint2*>(lds);
    uint16_t* dpl = reinterpret_cast<uint16_t*>(lds + 2 * lds_ct_words);
    for (uint32_t i = threadIdx.x; i < lds_ct_words; i += blockDim.x) ctl[i] = ((const uint2*)gbl(j0.coltab))[i];
    for (uint32_t i = threadIdx.x; i < dpre_n; i += blockDim.x) dpl[i] = gbl(j0.dpre)[i];
    T.ct = ctl;                                      // this variant runs only when the table fits
    T.dp = dpl;
    T.kg = nullptr;
    if (j0.kmod_fused && !kWide) {
      // after the column and residue tables, 8-byte aligned (the plan sized the region)
      const uint32_t off = ((2 * lds_ct_words + (dpre_n + 1) / 2) + 1) & ~1u;
      double* kgl = reinterpret_cast<double*>(lds + off);
      const uint32_t ng = gbl(j0.ctrl)->n_kgroups;
      for (uint32_t i = threadIdx.x; i < ng; i += blockDim.x) kgl[i] = (double)gbl(j0.kgroups)[i];
      T.kg = kgl;
    }
    __syncthreads();
  }
  LaneCount lc;
  lane_count_init(lc);
  ListReg lreg = {kNoChunk, 0u};
  uint32_t t_last = 0, ji_last = 0;                  // a lane's items only grow: resume the tier search
  for (uint64_t item = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; item < total;
       item += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t ji = 0;
    if constexpr (!kLds) {
      ji = ji_last;                                  // items only grow: resume the job search
      while (ji + 1 < n_jobs && job_item_base[ji + 1] <= item) ++ji;
      T.ct = gbl(jobs[ji].coltab);
      T.dp = gbl(jobs[ji].dpre);
      T.kg = gbl((const uint64_t*)jobs[ji].kgroups);
    }
    if (ji != ji_last) t_last = 0;
    ji_last = ji;
    // the LDS variant runs one job: its fields are uniform
    large_item<kLds, kSc, kG, kWide>(jobs[kLds ? 0 : ji], T, item - job_item_base[ji], t_last, lc, s_dec, lreg, lkey,
                                     s_sup);
    if constexpr (kSc == 2) list_sync(lreg, lkey);
  }
  if constexpr (kSc == 2) {
    // close the wavefront's last chunk; the LDS slot holds the latest state of all its lanes
    if ((threadIdx.x & (kWave - 1)) == 0) {
      const unsigned long long k = *reinterpret_cast<volatile unsigned long long*>(lkey);
      const uint32_t ch = (uint32_t)(k >> 32) - 1u;
      if (ch < kPoolFull) jobs[0].list_fill[ch] = (uint32_t)k;
    }
  }
  // counters: one atomic per workgroup, decade and counter, and the totals over the decades
  flush_dec(lc, s_dec);
  __syncthreads();
  if constexpr (kSc == 2) {
    if (threadIdx.x < kListSupers && s_sup[threadIdx.x]) atomicAdd(&jobs[0].list_super[threadIdx.x], s_sup[threadIdx.x]);
  }
  if (threadIdx.x < DC_COUNT * kDecades) {
    const uint32_t slot = threadIdx.x / kDecades, dc = threadIdx.x % kDecades;
    const unsigned long long v = s_dec[slot][dc];
    if (v && dec) atomicAdd(&dec[slot * kDecades + dc], v);
  }
  if (threadIdx.x < 4) {
    const uint32_t slot = threadIdx.x == 0 ? DC_RAW : threadIdx.x == 1 ? DC_HITS : threadIdx.x == 2 ? DC_SOLVES
                        : DC_LEVELS;
    unsigned long long v = 0;
    for (uint32_t i = 0; i < (uint32_t)kDecades; ++i) v += s_dec[slot][i];
    const uint32_t at = threadIdx.x == 0 ? D_LARGE_RAW : threadIdx.x == 1 ? D_LARGE_HITS
                      : threadIdx.x == 2 ? D_G_CALLS : D_G_LEVELS;
    if (v) atomicAdd(&diag[at], v);
  }
  if (lc.err) atomicOr(reinterpret_cast<unsigned long long*>(&diag[D_ERROR]), (unsigned long long)lc.err);
}

// ------------------------------------------------------------------------------------------
// Persistent batch kernel: the small- and large-branch work of many jobs in one launch.  The
// work is cut into tasks: every job's large-branch items in tasks of kBatchItems (four per lane),
// then every job's small-branch units (one task each).  k_batch_queue counts them on the device
// (the item counts come from k_prep_bounds) into a prefix table, and the workgroups of k_batch
// pop tasks from one device counter until none is left, so uneven jobs share the GPU without a
// launch per job.  A workgroup keeps the column table (and residue table) of its last job in LDS
// and reloads them only when the job changes.  The task's counters go to its job's totals.
// ------------------------------------------------------------------------------------------
// Task ranges: 2 n_jobs ranges (a job's large tasks or its small tasks) in one of three orders.
// Range q of order 0 (large first): q < n_jobs is job q's large tasks, then the small ones;
// order 1 (small first): the reverse; order 2 (by job): job q/2's large (q even) or small tasks.
__device__ __forceinline__ void batch_range(uint32_t q, uint32_t n_jobs, uint32_t order, uint32_t* job, bool* large) {
  if (order == 2) {
    *job = q >> 1;
    *large = (q & 1u) == 0;
  } else {
    *job = q < n_jobs ? q : q - n_jobs;
    *large = (q < n_jobs) == (order == 0);
  }
}

// tbase: 2 n_jobs + 1 entries, the first task of each range and the number of tasks.  A job's
// large tasks hold items_per_task items each, its small tasks one unit each.  Clears the task
// counter.
__global__ void k_batch_queue(const JobDev* __restrict__ jobs, uint32_t n_jobs, uint32_t items_per_task,
                              uint32_t order, uint64_t* __restrict__ tbase, unsigned long long* __restrict__ next) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t s = 0;
  for (uint32_t q = 0; q < 2 * n_jobs; ++q) {
    tbase[q] = s;
    uint32_t ji;
    bool large;
    batch_range(q, n_jobs, order, &ji, &large);
    const JobDev& j = jobs[ji];
    if (!j.n_m) continue;
    s += large ? (j.ctrl->n_items + items_per_task - 1) / items_per_task : (uint64_t)j.n_windows * j.n_slices;
  }
  tbase[2 * n_jobs] = s;
  *next = 0ull;
}

// The tier of item `local` of job j (the last tier whose first item is at or below it).
template <class CT>
__device__ __forceinline__ uint32_t tier_of(const CT& c, uint32_t n_tiers, uint64_t local) {
  uint32_t lo = 0, hi = n_tiers;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (c.tier_item_base[mid] <= local) lo = mid; else hi = mid;
  }
  return lo;
}

// Adds a workgroup's per-decade large-branch counters to a job's and clears them.
__device__ __forceinline__ void flush_job_decades(const JobDev& j, unsigned long long (*s_dec)[kDecades]) {
  unsigned long long* diag = j.ctrl->diag;
  unsigned long long* dec = &j.ctrl->dec[0][0];
  if (threadIdx.x < 4) {
    const uint32_t slot = threadIdx.x == 0 ? DC_RAW : threadIdx.x == 1 ? DC_HITS : threadIdx.x == 2 ? DC_SOLVES
                        : DC_LEVELS;
    unsigned long long v = 0;
    for (uint32_t i = 0; i < (uint32_t)kDecades; ++i) v += s_dec[slot][i];
    const uint32_t at = threadIdx.x == 0 ? D_LARGE_RAW : threadIdx.x == 1 ? D_LARGE_HITS
                      : threadIdx.x == 2 ? D_G_CALLS : D_G_LEVELS;
    if (v) atomicAdd(&diag[at], v);
  }
  __syncthreads();
  if (threadIdx.x < DC_COUNT * kDecades) {
    unsigned long long* sd = &s_dec[0][0];
    const unsigned long long v = sd[threadIdx.x];
    if (v) atomicAdd(&dec[threadIdx.x], v);
    sd[threadIdx.x] = 0ull;
  }
  __syncthreads();
}

template <int kSc, bool kG>
__global__ __launch_bounds__(256) void k_batch(const JobDev* __restrict__ jobs, uint32_t n_jobs,
                                               const uint64_t* __restrict__ tbase,
                                               unsigned long long* __restrict__ next, uint32_t lds_ct_words,
                                               uint32_t kg_off_words, uint32_t items_per_task, uint32_t order) {
  extern __shared__ uint32_t lds[];
  __shared__ unsigned long long s_dec[DC_COUNT][kDecades];
  __shared__ unsigned long long s_list[256 / kWave];   // list state (the list scatter is not used here)
  __shared__ uint32_t s_sup[kListSupers];
  __shared__ unsigned long long s_task;
  for (uint32_t i = threadIdx.x; i < DC_COUNT * kDecades; i += blockDim.x) (&s_dec[0][0])[i] = 0ull;
  if (threadIdx.x < 256 / kWave) s_list[threadIdx.x] = 0ull;
  if (threadIdx.x < kListSupers) s_sup[threadIdx.x] = 0u;
  const uint64_t total = tbase[2 * n_jobs];
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t ct_job = 0xffffffffu, dp_job = 0xffffffffu, kg_job = 0xffffffffu;
  LaneCount lc;
  lane_count_init(lc);
  ListReg lreg = {kNoChunk, 0u};
  for (;;) {
    if (threadIdx.x == 0) s_task = atomicAdd(next, 1ull);
    __syncthreads();
    const uint64_t task = s_task;
    __syncthreads();                                 // read before the next pop overwrites it
    if (task >= total) break;
    uint32_t lo = 0, hi = 2 * n_jobs;                // tbase[lo] <= task < tbase[hi]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (tbase[mid] <= task) lo = mid; else hi = mid;
    }
    uint32_t ji;
    bool large;
    batch_range(lo, n_jobs, order, &ji, &large);
    const JobDev& j = jobs[ji];
    const uint64_t local = task - tbase[lo];
    if (!large) {
      __builtin_amdgcn_s_setprio(0);                 // small tasks fill the cycles large ones leave
      unsigned long long n_pairs = 0, n_marks = 0;
      small_unit<false>(j, local, lds, lds_ct_words, ct_job == ji, n_pairs, n_marks);
      ct_job = ji;
      dp_job = kg_job = 0xffffffffu;                 // the tile overwrote the residue table and K's groups
      if (lane == 0) {
        if (n_pairs) atomicAdd(&j.ctrl->diag[D_SMALL_PAIRS], n_pairs);
        if (n_marks) atomicAdd(&j.ctrl->diag[D_SMALL_MARKS], n_marks);
      }
      continue;
    }
    // a large task: the job's tables in LDS (the plan guarantees they fit), then its items, at
    // the issue priority k_large takes over small-branch waves
    __builtin_amdgcn_s_setprio(1);
    uint2* ctl = reinterpret_cast<uint2*>(lds);
    uint16_t* dpl = reinterpret_cast<uint16_t*>(lds + 2 * lds_ct_words);
    if (ct_job != ji) {
      const uint32_t nct = (2 * j.sl + 1 + 31) / 32;
      for (uint32_t i = threadIdx.x; i < nct; i += blockDim.x) ctl[i] = ((const uint2*)gbl(j.coltab))[i];
    }
    if (dp_job != ji && j.d_small) {
      const uint32_t dn = (uint32_t)j.d;
      for (uint32_t i = threadIdx.x; i < dn; i += blockDim.x) dpl[i] = gbl(j.dpre)[i];
    }
    double* kgl = reinterpret_cast<double*>(lds + kg_off_words);
    if (j.kmod_fused && kg_job != ji) {              // K's groups, for K mod p formed per prime
      const uint32_t ng = gbl(j.ctrl)->n_kgroups;
      for (uint32_t i = threadIdx.x; i < ng; i += blockDim.x) kgl[i] = (double)gbl(j.kgroups)[i];
      kg_job = ji;
    }
    ct_job = dp_job = ji;
    __syncthreads();
    LargeTables<true> T;
    T.ct = ctl;
    T.dp = dpl;
    T.kg = j.kmod_fused ? kgl : nullptr;             // else the job reads K mod p from its tables
    const auto& c = *gbl(j.ctrl);
    const uint64_t n_items = c.n_items;
    const uint64_t first = local * items_per_task;
    uint32_t t_last = tier_of(c, j.n_tiers, first);
    for (uint32_t k = 0; k < items_per_task; k += 256u) {
      const uint64_t item = first + k + threadIdx.x;
      if (item < n_items)
        large_item<true, kSc, kG>(j, T, item, t_last, lc, s_dec, lreg, s_list + threadIdx.x / kWave, s_sup);
    }
    flush_dec(lc, s_dec);
    lc.cur_dec = kDecades;
    if (lc.err) {
      atomicOr(reinterpret_cast<unsigned long long*>(&j.ctrl->diag[D_ERROR]), (unsigned long long)lc.err);
      lc.err = 0;
    }
    __syncthreads();
    flush_job_decades(j, s_dec);
  }
}

// Folds the byte counters of large-prime hits into the bitmap and the counts, one wavefront per
// row (each lane takes 32 columns = one bitmap word at a time), and clears them for the next call.
// Every counter is below 256 (the plan admits the counters only when no number of the interval
// can have more distinct prime factors above the threshold), so the byte sums never carry.
// One 32-byte group of counters (32 column slots): its bitmap word and the sum of its counts.
__device__ __forceinline__ uint32_t fold_group(const uint4 a, const uint4 b, uint32_t* sum) {
  const uint32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  uint32_t bits = 0, s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t x = v[q];
    bits |= (((x & 0xffu) ? 1u : 0u) | ((x & 0xff00u) ? 2u : 0u) | ((x & 0xff0000u) ? 4u : 0u) |
             ((x & 0xff000000u) ? 8u : 0u)) << (4 * q);
    const uint32_t h = (x & 0x00ff00ffu) + ((x >> 8) & 0x00ff00ffu);   // two 16-bit pair sums
    s += (h & 0xffffu) + (h >> 16);
  }
  *sum += s;
  return bits;
}

// One wavefront per row; each lane loads two 32-byte groups before folding either, so twice
// the bytes are in flight per wavefront.
__global__ __launch_bounds__(256) void k_fold_bytes(const JobDev* __restrict__ jobs) {
  const JobDev& j = jobs[blockIdx.y];
  if (!j.hitbytes) return;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t waves = blockDim.x / kWave;
  const bool clear = !j.fold_keep;
  const uint32_t rw = j.row_words;
  for (uint64_t row = blockIdx.x * (uint64_t)waves + threadIdx.x / kWave; row < j.n_m;
       row += (uint64_t)gridDim.x * waves) {
    uint4* __restrict__ src = (uint4*)(gbl(j.hitbytes) + row * rw * 32ull);
    const gptr<uint32_t> dst = gbl(j.bitmap) + row * rw;
    uint32_t sum = 0;                       // at most 255 x 32 per group a lane folds
    for (uint32_t w0 = lane; w0 < rw; w0 += 2 * kWave) {
      const uint32_t w1 = w0 + kWave;
      const bool has1 = w1 < rw;
      const uint4 a0 = src[2 * w0], b0 = src[2 * w0 + 1];
      uint4 a1 = make_uint4(0, 0, 0, 0), b1 = make_uint4(0, 0, 0, 0);
      if (has1) {
        a1 = src[2 * w1];
        b1 = src[2 * w1 + 1];
      }
      const uint32_t bits0 = fold_group(a0, b0, &sum);
      const uint32_t bits1 = fold_group(a1, b1, &sum);
      if (bits0) {
        if (clear) {
          src[2 * w0] = make_uint4(0, 0, 0, 0);
          src[2 * w0 + 1] = make_uint4(0, 0, 0, 0);
        }
        dst[w0] |= bits0;
      }
      if (bits1) {
        if (clear) {
          src[2 * w1] = make_uint4(0, 0, 0, 0);
          src[2 * w1 + 1] = make_uint4(0, 0, 0, 0);
        }
        dst[w1] |= bits1;
      }
    }
    const unsigned long long tot = wave_sum_u64(sum);
    if (lane == 0 && tot) gbl(j.counts)[row] += (uint32_t)tot;
  }
}

// Clears the byte buffer of every job that has one.
__global__ __launch_bounds__(256) void k_zero_bytes(const JobDev* __restrict__ jobs) {
  const JobDev& j = jobs[blockIdx.y];
  if (!j.hitbytes) return;
  const uint64_t n = j.n_m * (uint64_t)j.row_words * 8;
  const gptr<uint32_t> p = (gptr<uint32_t>)gbl(j.hitbytes);
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ------------------------------------------------------------------------------------------
// Grouping of the list scatter.  Cells are (row << cell_shift) | col, buckets are 2^k rows and
// groups are 2^g buckets, so bucket = cell >> bkt_shift and group = cell >> (bkt_shift + g).  The
// large branch counted the cells of each group (list_super); a scan gives the groups' ranges; the
// first pass moves every cell of the pool to its group's range and counts the cells of each
// bucket; a scan gives the buckets' ranges; the second pass moves the cells of each group to their
// buckets; then one block per bucket ORs its cells into an LDS tile of the bucket's rows and merges
// the tile into the bitmap and the counts (the block owns those rows).  Cells of a bucket come in
// no particular order: OR and sums do not depend on it.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t list_n_chunks(const JobDev& j) {
  const unsigned long long c = *j.list_cursor;
  return c < j.list_chunks ? c : j.list_chunks;
}

// list_super layout: counts [kListSupers + 1], bases [kListSupers + 1], cursors [kListSupers + 1].
constexpr uint32_t kSupStride = kListSupers + 1;

// Bases and cursors of the groups from the large branch's counts (one wavefront).
__global__ __launch_bounds__(64) void k_list_scan1(const JobDev* __restrict__ jobs) {
  const JobDev& j = jobs[0];
  uint32_t* cnt = j.list_super;
  uint32_t* base = cnt + kSupStride;
  uint32_t* cur = base + kSupStride;
  const uint32_t t = threadIdx.x;
  const uint32_t v = t < kListSupers ? cnt[t] : 0u;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, kWave);
    if ((int)t >= o) x += y;
  }
  if (t < kListSupers) {
    base[t] = x - v;
    cur[t] = x - v;
  }
  if (t == kWave - 1) base[kListSupers] = x;
}

constexpr uint32_t kPartBatch = 4096;   // cells per batch of the partition passes (16 per thread)

// One batch of a partition pass: up to kPartBatch cells src[0, nf) are ranked per key in LDS,
// each key with cells in the batch reserves a run of its output range with one atomic on its
// global cursor, the cells are placed by key in an LDS stage, and consecutive threads write each
// key's run (contiguous stores).  cnt (n_keys <= 256 words) is zero on entry and on exit.  With
// hist2, each cell also adds one to the LDS counter of its bucket (cell >> bsh).
template <class KeyOf>
__device__ __forceinline__ void part_batch(const uint32_t* __restrict__ src, uint32_t nf, uint32_t n_keys,
                                           KeyOf key_of, uint32_t* cnt, uint32_t* start, uint32_t* gofs,
                                           uint32_t* stg, uint32_t* __restrict__ gcur, uint32_t* __restrict__ dst,
                                           uint32_t* hist2, uint32_t bsh) {
  constexpr uint32_t kPer = kPartBatch / 256;
  uint32_t cell[kPer], rk[kPer];
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t i = threadIdx.x + 256u * k;
    cell[k] = i < nf ? src[i] : 0u;
  }
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t i = threadIdx.x + 256u * k;
    if (i < nf) {
      rk[k] = atomicAdd(&cnt[key_of(cell[k])], 1u);
      if (hist2) atomicAdd(&hist2[cell[k] >> bsh], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x < kWave) {
    // the first wavefront scans the counts (up to 4 consecutive keys per lane) and reserves the runs
    const uint32_t lane = threadIdx.x;
    const uint32_t per = (n_keys + kWave - 1) / kWave;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t key = lane * per + q;
      v[q] = (q < per && key < n_keys) ? cnt[key] : 0u;
      sum += v[q];
    }
    uint32_t x = sum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, kWave);
      if ((int)lane >= o) x += y;
    }
    uint32_t ex = x - sum;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t key = lane * per + q;
      if (q < per && key < n_keys) {
        start[key] = ex;
        if (v[q]) gofs[key] = atomicAdd(&gcur[key], v[q]);
        ex += v[q];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t i = threadIdx.x + 256u * k;
    if (i < nf) stg[start[key_of(cell[k])] + rk[k]] = cell[k];
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nf; i += 256u) {
    const uint32_t c = stg[i];
    const uint32_t key = key_of(c);
    dst[gofs[key] + (i - start[key])] = c;
  }
  for (uint32_t q = threadIdx.x; q < n_keys; q += 256u) cnt[q] = 0u;
  __syncthreads();
}

// First pass: the pool's chunks -> their groups' ranges of list_sorted, and the bucket counts.
// Each block takes kListChunksPerBlock chunks; its bucket counts (n_bkt words of dynamic LDS)
// reach bkt_count with one atomic per bucket at its end.
__global__ __launch_bounds__(256) void k_list_part1(const JobDev* __restrict__ jobs) {
  const JobDev& j = jobs[0];
  extern __shared__ uint32_t hist2[];
  __shared__ uint32_t cnt[kListSupers], start[kListSupers], gofs[kListSupers], fills[kListChunksPerBlock];
  __shared__ uint32_t stg[kPartBatch];
  const uint64_t n_chunks = list_n_chunks(j);
  const uint64_t c0 = blockIdx.x * (uint64_t)kListChunksPerBlock;
  if (c0 >= n_chunks) return;
  const uint32_t nc = (uint32_t)min<uint64_t>(kListChunksPerBlock, n_chunks - c0);
  const uint32_t n_bkt = j.n_bkt;
  for (uint32_t i = threadIdx.x; i < n_bkt; i += blockDim.x) hist2[i] = 0u;
  if (threadIdx.x < kListSupers) cnt[threadIdx.x] = 0u;
  for (uint32_t i = threadIdx.x; i < nc; i += blockDim.x) fills[i] = min(j.list_fill[c0 + i], kListChunk);
  __syncthreads();
  const uint32_t ssh = j.bkt_shift + j.super_shift, bsh = j.bkt_shift;
  uint32_t* cur = j.list_super + 2 * kSupStride;
  auto key_of = [ssh](uint32_t cell) { return cell >> ssh; };
  for (uint32_t c = 0; c < nc; ++c)
    part_batch(j.list_pool + (c0 + c) * kListChunk, fills[c], kListSupers, key_of, cnt, start, gofs, stg, cur,
               j.list_sorted, hist2, bsh);
  for (uint32_t i = threadIdx.x; i < n_bkt; i += blockDim.x)
    if (hist2[i]) atomicAdd(&j.bkt_count[i], hist2[i]);
}

// Exclusive scan of n_bkt <= kMaxBuckets bucket counts by one block of 1024 threads: the buckets'
// bases and cursors.
__global__ __launch_bounds__(1024) void k_list_scan(const JobDev* __restrict__ jobs) {
  const JobDev& j = jobs[0];
  __shared__ uint32_t part[1024];
  constexpr uint32_t per = kMaxBuckets / 1024;
  uint32_t v[per];
  uint32_t sum = 0;
#pragma unroll
  for (uint32_t k = 0; k < per; ++k) {
    const uint32_t i = threadIdx.x * per + k;
    v[k] = i < j.n_bkt ? j.bkt_count[i] : 0u;
    sum += v[k];
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (uint32_t off = 1; off < 1024; off <<= 1) {
    const uint32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - sum;
#pragma unroll
  for (uint32_t k = 0; k < per; ++k) {
    const uint32_t i = threadIdx.x * per + k;
    if (i < j.n_bkt) {
      j.bkt_base[i] = run;
      j.bkt_cursor[i] = run;
    }
    run += v[k];
  }
  if (threadIdx.x == 1023) j.bkt_base[j.n_bkt] = part[1023];
}

// Second pass: each group's range of list_sorted -> its buckets' ranges, into list_pool (free by
// now).  Block (x, g) takes pieces x, x + gridDim.x, ... of kListPiece cells of group g.
__global__ __launch_bounds__(256) void k_list_part2(const JobDev* __restrict__ jobs) {
  const JobDev& j = jobs[0];
  __shared__ uint32_t cnt[kListMaxPerSuper], start[kListMaxPerSuper], gofs[kListMaxPerSuper];
  __shared__ uint32_t stg[kPartBatch];
  const uint32_t g = j.bkt_per_super;
  const uint32_t sup = blockIdx.y;
  const uint32_t b0 = sup * g;
  if (b0 >= j.n_bkt) return;
  const uint32_t nk = min(b0 + g, j.n_bkt) - b0;
  const uint32_t* sbase = j.list_super + kSupStride;
  const uint32_t lo = sbase[sup], hi = sbase[sup + 1];
  const uint32_t bsh = j.bkt_shift;
  for (uint32_t i = threadIdx.x; i < nk; i += blockDim.x) cnt[i] = 0u;
  __syncthreads();
  auto key_of = [bsh, b0](uint32_t cell) { return (cell >> bsh) - b0; };
  for (uint64_t p0 = lo + (uint64_t)blockIdx.x * kListPiece; p0 < hi; p0 += (uint64_t)gridDim.x * kListPiece) {
    const uint32_t p1 = (uint32_t)min<uint64_t>(p0 + kListPiece, hi);
    for (uint32_t e = (uint32_t)p0; e < p1; e += kPartBatch)
      part_batch(j.list_sorted + e, min(kPartBatch, p1 - e), nk, key_of, cnt, start, gofs, stg, j.bkt_cursor + b0,
                 j.list_pool, nullptr, 0u);
  }
}

__global__ __launch_bounds__(256) void k_list_apply(const JobDev* __restrict__ jobs) {
  const JobDev& j = jobs[0];
  extern __shared__ uint32_t tile[];   // bkt_rows x row_words words, then bkt_rows counts
  const uint32_t b = blockIdx.x;
  if (b >= j.n_bkt) return;
  const uint64_t row0 = (uint64_t)b * j.bkt_rows;
  const uint32_t rows = (uint32_t)min<uint64_t>(j.bkt_rows, j.n_m - row0);
  const uint32_t words = rows * j.row_words;
  uint32_t* cnt = tile + j.bkt_rows * j.row_words;
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) tile[i] = 0;
  for (uint32_t i = threadIdx.x; i < rows; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  const uint32_t e0 = j.bkt_base[b], e1 = j.bkt_base[b + 1];
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const uint32_t cell = j.list_pool[e];
    const uint32_t row = cell >> j.cell_shift;
    const uint32_t col = cell & ((1u << j.cell_shift) - 1u);
    const uint32_t lr = row - (uint32_t)row0;
    if (lr < rows && col < j.n_x) {
      atomicOr(&tile[lr * j.row_words + (col >> 5)], 1u << (col & 31));
      atomicAdd(&cnt[lr], 1u);
    }
  }
  __syncthreads();
  uint32_t* __restrict__ dst = j.bitmap + row0 * j.row_words;
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) {
    const uint32_t v = tile[i];
    if (v) dst[i] |= v;
  }
  for (uint32_t i = threadIdx.x; i < rows; i += blockDim.x)
    if (cnt[i]) j.counts[row0 + i] += cnt[i];
}

// ------------------------------------------------------------------------------------------
// Scatter-rate probe: the device's rate of the memory operations the hit scatters issue, at
// pseudo-random 32-bit words generated in registers (a 64-bit mixing hash of the operation
// index), so that no index is ever loaded.  op 0: atomic add of 1 at device scope (no return);
// op 1: plain 4-byte store; op 2: atomic add of 1 into LDS (a 64 KB table per workgroup, the
// rate of the LDS-tile scatters).  slices > 1: the buffer is cut into `slices` equal ranges and
// a workgroup only touches range (XCC id mod slices), the id read from the hardware, which keeps
// each range in the L2 of the one XCD that uses it.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 31;
  x *= 0x7fb5d329728ea185ull;
  x ^= x >> 27;
  x *= 0x81dadef4bc2dd44dull;
  x ^= x >> 33;
  return x;
}

__global__ __launch_bounds__(256) void k_probe_scatter(uint32_t* __restrict__ buf, uint64_t words, uint64_t n_ops,
                                                       uint32_t slices, uint32_t op, uint64_t seed) {
  __shared__ uint32_t tab[16384];
  uint64_t range = words, base = 0;
  if (slices > 1) {
    const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u;   // HW_REG_XCC_ID
    range = words / slices;
    base = (uint64_t)(xcc % slices) * range;
  }
  if (op == 2) {
    for (uint32_t i = threadIdx.x; i < 16384; i += blockDim.x) tab[i] = 0;
    __syncthreads();
    range = 16384;
    base = 0;
  }
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t acc = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_ops; i += stride) {
    const uint64_t h = mix64(i ^ seed);
    const uint64_t w = base + __umul64hi(h, range);          // uniform in [base, base + range)
    if (op == 0) atomicAdd(&buf[w], 1u);
    else if (op == 1) buf[w] = (uint32_t)h | 1u;
    else atomicAdd(&tab[w], 1u);
  }
  if (op == 2) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < 16384; i += blockDim.x) acc += tab[i];
    acc = wave_sum_u32(acc);
    if ((threadIdx.x & (kWave - 1)) == 0 && acc) atomicAdd(&buf[0], acc);   // the ops, for the caller's check
  }
}

// ------------------------------------------------------------------------------------------
// launch wrappers (host)
// ------------------------------------------------------------------------------------------
static thread_local char g_last_error[256];

// Records the failing kernel's name with the runtime's message; returns the error.
static hipError_t note(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) snprintf(g_last_error, sizeof g_last_error, "%s: %s", what, hipGetErrorString(e));
  return e;
}

const char* last_error_detail() { return g_last_error; }

hipError_t record_launch(const char* what) { return note(what); }

hipError_t launch_write_job(const JobDev& jd, JobDev* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_write_job, dim3(1), dim3(1), 0, s, jd, dst); { hipError_t e_ = note("k_write_job"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_upload(void* dst, const void* src, uint64_t bytes, hipStream_t s) {
  const uint8_t* in = static_cast<const uint8_t*>(src);
  uint8_t* out = static_cast<uint8_t*>(dst);
  for (uint64_t at = 0; at < bytes; at += sizeof(UploadChunk)) {
    UploadChunk c;
    const uint32_t n = (uint32_t)((bytes - at) < sizeof(c) ? (bytes - at) : sizeof(c));
    memcpy(c.bytes, in + at, n);
    hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, c, out + at, n); { hipError_t e_ = note("k_upload"); if (e_ != hipSuccess) return e_; }
  }
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p, n, v); { hipError_t e_ = note("k_fill_u32"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_zero_ctrl(JobCtrl* c, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ctrl, dim3(1), dim3(256), 0, s, c); { hipError_t e_ = note("k_zero_ctrl"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_primes(uint64_t lim, const PrimeWs& pw, hipStream_t s) {
  return launch_primes_range(0, lim, pw, s);
}

hipError_t launch_primes_range(uint64_t seg0, uint64_t lim, const PrimeWs& pw, hipStream_t s) {
  const uint64_t n_seg = (lim >> kSegLog) + 1 - seg0;
  uint32_t blocks = (uint32_t)(n_seg < 8192 ? n_seg : 8192);
  const uint32_t seg_blocks = (uint32_t)(n_seg < (1ull << 31) ? n_seg : (1ull << 31));   // one per segment
  if (pw.isq && lim >= (1ull << 42)) {
    // level 2: the primes up to sqrt(lim) with the LDS-sieved base, then the segments with them
    PrimeWs p2;
    p2.base = pw.base;
    p2.n_base = pw.n_base;
    p2.flags = pw.flags2;
    p2.seg_count = pw.seg_count2;
    p2.seg_off = pw.seg_off2;
    p2.primes = pw.base2;
    p2.n_primes = pw.n_base2;
    p2.cap = pw.cap2;
    hipError_t e = launch_primes_range(0, pw.isq, p2, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sieve_segments<true, uint64_t, uint64_t>), dim3(seg_blocks), dim3(kSieveThreads), 0, s, lim, seg0, n_seg,
                       (const uint64_t*)pw.base2, (const uint64_t*)pw.n_base2, pw.flags, pw.seg_count);
    { hipError_t e_ = note("k_sieve_segments<wide>"); if (e_ != hipSuccess) return e_; }
  } else {
    hipLaunchKernelGGL(k_base_primes, dim3(1), dim3(1024), 0, s, lim, pw.base, pw.n_base); { hipError_t e_ = note("k_base_primes"); if (e_ != hipSuccess) return e_; }
    hipLaunchKernelGGL((k_sieve_segments<false, uint32_t, uint32_t>), dim3(seg_blocks), dim3(kSieveThreads), 0, s, lim, seg0, n_seg,
                       (const uint32_t*)pw.base, (const uint32_t*)pw.n_base, pw.flags, pw.seg_count);
    { hipError_t e_ = note("k_sieve_segments"); if (e_ != hipSuccess) return e_; }
  }
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, pw.seg_count, n_seg, pw.seg_off, pw.n_primes); { hipError_t e_ = note("k_scan_counts"); if (e_ != hipSuccess) return e_; }
  hipLaunchKernelGGL(k_compact_primes, dim3(blocks), dim3(256), 0, s, seg0, n_seg, pw.flags, pw.seg_off,
                     pw.primes, pw.cap); { hipError_t e_ = note("k_compact_primes"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_chunk_bounds(JobDev* jobs, hipStream_t s) {
  hipLaunchKernelGGL(k_chunk_bounds, dim3(1, 1), dim3(64), 0, s, jobs);
  return note("k_chunk_bounds");
}

hipError_t launch_prep_tables(JobDev* jobs, uint32_t n_jobs, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_tables, dim3(1, n_jobs), dim3(64), 0, s, jobs); { hipError_t e_ = note("k_prep_tables"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_kmod(const JobDev* jobs, uint32_t n_jobs, uint64_t* lim_base, uint64_t total_cap, int n_cu,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_lim_scan, dim3(1), dim3(64), 0, s, jobs, n_jobs, lim_base); { hipError_t e_ = note("k_lim_scan"); if (e_ != hipSuccess) return e_; }
  uint64_t blocks = (total_cap + 255) / 256;
  uint64_t maxb = (uint64_t)n_cu * 32;
  if (blocks > maxb) blocks = maxb;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_kmod, dim3((uint32_t)blocks), dim3(256), 0, s, jobs, n_jobs, (const uint64_t*)lim_base); { hipError_t e_ = note("k_kmod"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_fill_jobs(const JobDev* jobs, uint32_t n_jobs, uint64_t max_words, hipStream_t s) {
  uint64_t blocks = (max_words + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_fill_jobs, dim3((uint32_t)blocks, n_jobs), dim3(256), 0, s, jobs); { hipError_t e_ = note("k_fill_jobs"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_zero_ctrls(const JobDev* jobs, uint32_t n_jobs, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ctrls, dim3(1, n_jobs), dim3(256), 0, s, jobs); { hipError_t e_ = note("k_zero_ctrls"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_kmod_list(const uint64_t* primes, uint64_t n, const uint64_t* groups, uint32_t ng,
                            uint64_t* out, int n_cu, hipStream_t s) {
  uint64_t blocks = (n + 255) / 256;
  uint64_t maxb = (uint64_t)n_cu * 32;
  if (blocks > maxb) blocks = maxb;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_kmod_list, dim3((uint32_t)blocks), dim3(256), 0, s, primes, n, groups, ng, out); { hipError_t e_ = note("k_kmod_list"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_rows_cols(const JobDev* jobs, uint32_t n_jobs, uint64_t max_m_inc, uint32_t max_sl, int n_cu,
                            hipStream_t s) {
  const uint64_t nb = (max_m_inc + kRowBlock - 1) / kRowBlock;
  uint32_t blocks = (uint32_t)(nb < (uint64_t)n_cu * 16 ? nb : (uint64_t)n_cu * 16);
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_rows_count, dim3(blocks, n_jobs), dim3(256), 0, s, jobs); { hipError_t e_ = note("k_rows_count"); if (e_ != hipSuccess) return e_; }
  hipLaunchKernelGGL(k_rows_scan, dim3(1, n_jobs), dim3(1024), 0, s, jobs); { hipError_t e_ = note("k_rows_scan"); if (e_ != hipSuccess) return e_; }
  hipLaunchKernelGGL(k_rows_write, dim3(blocks, n_jobs), dim3(1024), 0, s, jobs); { hipError_t e_ = note("k_rows_write"); if (e_ != hipSuccess) return e_; }
  const uint32_t nwords = (2 * max_sl + 1 + 31) / 32;
  uint32_t cb = (nwords * 32 + 255) / 256;
  if (cb > 4096) cb = 4096;
  hipLaunchKernelGGL(k_cols_mask, dim3(cb, n_jobs), dim3(256), 0, s, jobs); { hipError_t e_ = note("k_cols_mask"); if (e_ != hipSuccess) return e_; }
  hipLaunchKernelGGL(k_cols_prefix, dim3(1, n_jobs), dim3(1024), 0, s, jobs); { hipError_t e_ = note("k_cols_prefix"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_dpattern(const JobDev* jobs, uint32_t n_jobs, uint32_t max_phi, uint32_t max_row_words,
                           hipStream_t s) {
  if (max_phi == 0) return hipSuccess;
  const uint32_t blocks = max_phi < 1024 ? max_phi : 1024;
  hipLaunchKernelGGL(k_dpattern, dim3(blocks, n_jobs), dim3(256), max_row_words * 4u, s, jobs); { hipError_t e_ = note("k_dpattern"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_fold_bytes(const JobDev* jobs, uint32_t n_jobs, uint64_t max_rows, int n_cu, hipStream_t s) {
  uint64_t blocks = (max_rows + 3) / 4;
  if (blocks > (uint64_t)n_cu * 16) blocks = (uint64_t)n_cu * 16;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_fold_bytes, dim3((uint32_t)blocks, n_jobs), dim3(256), 0, s, jobs); { hipError_t e_ = note("k_fold_bytes"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_zero_bytes(const JobDev* jobs, uint32_t n_jobs, uint64_t max_words, int n_cu, hipStream_t s) {
  uint64_t blocks = (max_words * 8 + 255) / 256;
  if (blocks > (uint64_t)n_cu * 16) blocks = (uint64_t)n_cu * 16;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_zero_bytes, dim3((uint32_t)blocks, n_jobs), dim3(256), 0, s, jobs); { hipError_t e_ = note("k_zero_bytes"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_prep_bounds(JobDev* jobs, uint32_t n_jobs, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_bounds, dim3(1, n_jobs), dim3(64), 0, s, jobs); { hipError_t e_ = note("k_prep_bounds"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_items_scan(const JobDev* jobs, uint32_t n_jobs, uint64_t* base, hipStream_t s) {
  hipLaunchKernelGGL(k_items_scan, dim3(1), dim3(64), 0, s, jobs, n_jobs, base); { hipError_t e_ = note("k_items_scan"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_small(const JobDev* jobs, uint32_t n_jobs, uint64_t total_units, uint32_t lds_bytes,
                        uint32_t lds_ct_words, uint32_t blocks, hipStream_t s, bool hit_rows) {
  if (total_units == 0) return hipSuccess;
  if (hit_rows)
    hipLaunchKernelGGL(k_small<true>, dim3(blocks), dim3(256), lds_bytes, s, jobs, n_jobs, total_units, lds_ct_words);
  else
    hipLaunchKernelGGL(k_small<false>, dim3(blocks), dim3(256), lds_bytes, s, jobs, n_jobs, total_units, lds_ct_words);
  { hipError_t e_ = note("k_small"); if (e_ != hipSuccess) return e_; }
  return hipGetLastError();
}

hipError_t launch_large(const JobDev* jobs, uint32_t n_jobs, const uint64_t* job_item_base,
                        unsigned long long* diag, unsigned long long* dec, uint32_t blocks, uint32_t lds_bytes,
                        uint32_t lds_ct_words, uint32_t dpre_n, uint32_t scatter_kind, uint32_t large_mode,
                        hipStream_t s, bool wide) {
  if (n_jobs != 1 && scatter_kind == 2) scatter_kind = 0;   // the list serves single jobs only
  if (n_jobs != 1) wide = false;                            // (the 64-bit path serves single jobs)
  const bool lds = lds_bytes && lds_ct_words && n_jobs == 1;
#define LARGE_CASE(L, K, G, W)                                                                                 \
  hipLaunchKernelGGL((k_large<L, K, G, W>), dim3(blocks), dim3(256), L ? lds_bytes : 0u, s, jobs, n_jobs,       \
                     job_item_base, diag, dec, L ? lds_ct_words : 0u, L ? dpre_n : 0u)
#define LARGE_MODES(L, K)                                  \
  do {                                                     \
    if (wide) {                                            \
      if (large_mode == 0) LARGE_CASE(L, K, true, true);   \
      else LARGE_CASE(L, K, false, true);                  \
    } else {                                               \
      if (large_mode == 0) LARGE_CASE(L, K, true, false);  \
      else LARGE_CASE(L, K, false, false);                 \
    }                                                      \
  } while (0)
  if (lds) {
    if (scatter_kind == 2) LARGE_MODES(true, 2);
    else if (scatter_kind == 1) LARGE_MODES(true, 1);
    else LARGE_MODES(true, 0);
  } else {
    if (scatter_kind == 2) LARGE_MODES(false, 2);
    else if (scatter_kind == 1) LARGE_MODES(false, 1);
    else LARGE_MODES(false, 0);
  }
#undef LARGE_MODES
#undef LARGE_CASE
  return note(lds ? "k_large<lds>" : "k_large");
}

hipError_t launch_probe_scatter(uint32_t* buf, uint64_t words, uint64_t n_ops, uint32_t slices, uint32_t op,
                                uint64_t seed, int n_cu, hipStream_t s) {
  hipLaunchKernelGGL(k_probe_scatter, dim3((uint32_t)n_cu * 32u), dim3(256), 0, s, buf, words, n_ops, slices, op, seed);
  return note("k_probe_scatter");
}

hipError_t launch_batch_persistent(const JobDev* jobs, uint32_t n_jobs, uint64_t* tbase, unsigned long long* next,
                                   uint32_t blocks, uint32_t lds_bytes, uint32_t lds_ct_words, uint32_t kg_off_words,
                                   uint32_t scatter_kind, uint32_t large_mode, uint32_t items_per_task, uint32_t order,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_batch_queue, dim3(1), dim3(64), 0, s, jobs, n_jobs, items_per_task, order, tbase, next);
  { hipError_t e_ = note("k_batch_queue"); if (e_ != hipSuccess) return e_; }
#define BATCH_CASE(K, G) \
  hipLaunchKernelGGL((k_batch<K, G>), dim3(blocks), dim3(256), lds_bytes, s, jobs, n_jobs, (const uint64_t*)tbase, next, \
                     lds_ct_words, kg_off_words, items_per_task, order)
  if (scatter_kind == 1) {
    if (large_mode == 0) BATCH_CASE(1, true); else BATCH_CASE(1, false);
  } else {
    if (large_mode == 0) BATCH_CASE(0, true); else BATCH_CASE(0, false);
  }
#undef BATCH_CASE
  return note("k_batch");
}

hipError_t launch_list_group(const JobDev* job, uint64_t list_chunks, uint32_t n_bkt, uint32_t bkt_rows,
                             uint32_t super_shift, uint32_t row_words, hipStream_t s) {
  if (n_bkt == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)((list_chunks + kListChunksPerBlock - 1) / kListChunksPerBlock);
  hipLaunchKernelGGL(k_list_scan1, dim3(1), dim3(kWave), 0, s, job);
  { hipError_t e_ = note("k_list_scan1"); if (e_ != hipSuccess) return e_; }
  if (blocks) {
    hipLaunchKernelGGL(k_list_part1, dim3(blocks), dim3(256), n_bkt * 4u, s, job);
    { hipError_t e_ = note("k_list_part1"); if (e_ != hipSuccess) return e_; }
  }
  hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(1024), 0, s, job);
  { hipError_t e_ = note("k_list_scan"); if (e_ != hipSuccess) return e_; }
  if (blocks) {
    const uint32_t n_sup = (n_bkt + (1u << super_shift) - 1) >> super_shift;
    hipLaunchKernelGGL(k_list_part2, dim3(kListPart2X, n_sup), dim3(256), 0, s, job);
    { hipError_t e_ = note("k_list_part2"); if (e_ != hipSuccess) return e_; }
  }
  hipLaunchKernelGGL(k_list_apply, dim3(n_bkt), dim3(256), (bkt_rows * row_words + bkt_rows) * 4u, s, job);
  return note("k_list_apply");
}

}  // namespace cs

// Probable-prime stage after the sieve: a strong test to base 2 per candidate on the GPU, and the
// search for the nearest probable prime below and above each N = m*K among the unmarked columns
// of a sieved row (Section 2: after sieving, the survivors are tested walking away from N until
// both surrounding primes are found; Section 2.2: a probabilistic test, as the first half of BPSW).
//
// Arithmetic: one lane per candidate, numbers of NL 32-bit limbs (NL fixed per instantiation),
// Montgomery squaring by coarsely integrated operand scanning.  The multiplicand and the modulus
// live in registers (compile-time limb indices); the multiplier limb of the outer loop is read
// from this lane's column of LDS (lane-strided, conflict-free), so only the inner loops are
// unrolled and the code of one squaring stays a few KB.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/csieve.h"
#include "device.h"
#include "launch.h"
#include "plan.h"

namespace cs {
namespace {

constexpr int kPrpBlock = 256;
// Candidates per open side and round: at least kSurroundB0, and enough to fill the device once
// (the test kernel's resident candidates: a round of fewer costs as much), at most kSurroundBMax.
// Small rounds waste few tests past each side's first probable prime.
constexpr uint32_t kSurroundB0 = 2;
constexpr uint32_t kSurroundBMax = 1024;
constexpr uint64_t kSurroundSlotsMin = 1u << 18;

// out = v - n if (v >= n or hi_set) else v, for v < 2n given as NL limbs plus the bit hi_set.
// The comparison runs as a borrow-only pass and the subtraction of n & mask as a second pass, so
// no second NL-limb temporary is live.
template <int NL>
__device__ __forceinline__ void sub_if_ge(const uint32_t* v, bool hi_set, const uint32_t (&n)[NL], uint32_t (&out)[NL]) {
  uint32_t br = 0;
#pragma unroll
  for (int j = 0; j < NL; ++j) br = (uint32_t)(((uint64_t)v[j] - n[j] - br) >> 32) & 1u;
  const uint32_t mask = (hi_set || br == 0) ? 0xffffffffu : 0u;
  br = 0;
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const uint64_t d = (uint64_t)v[j] - (n[j] & mask) - br;
    out[j] = (uint32_t)d;
    br = (uint32_t)(d >> 32) & 1u;
  }
}

// a = a*a/R mod n, R = 2^(32 NL); requires a < n, n odd; b = this lane's LDS column.
template <int NL>
__device__ __forceinline__ void mont_sqr(uint32_t (&a)[NL], const uint32_t (&n)[NL], uint32_t ninv,
                                         uint32_t* __restrict__ b) {
#pragma unroll
  for (int j = 0; j < NL; ++j) b[j * kPrpBlock] = a[j];
  uint32_t t[NL + 2];
#pragma unroll
  for (int j = 0; j < NL + 2; ++j) t[j] = 0;
#pragma unroll 1
  for (int i = 0; i < NL; ++i) {
    const uint32_t bi = b[i * kPrpBlock];
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < NL; ++j) {                 // t += a * b_i
      const uint64_t s = (uint64_t)a[j] * bi + t[j] + c;
      t[j] = (uint32_t)s;
      c = (uint32_t)(s >> 32);
    }
    uint64_t s = (uint64_t)t[NL] + c;
    t[NL] = (uint32_t)s;
    t[NL + 1] = (uint32_t)(s >> 32);
    const uint32_t q = t[0] * ninv;                // t + q n = 0 (mod 2^32)
    s = (uint64_t)q * n[0] + t[0];
    c = (uint32_t)(s >> 32);
#pragma unroll
    for (int j = 1; j < NL; ++j) {                 // t = (t + q n) / 2^32
      s = (uint64_t)q * n[j] + t[j] + c;
      t[j - 1] = (uint32_t)s;
      c = (uint32_t)(s >> 32);
    }
    s = (uint64_t)t[NL] + c;
    t[NL - 1] = (uint32_t)s;
    t[NL] = t[NL + 1] + (uint32_t)(s >> 32);
  }
  sub_if_ge<NL>(t, t[NL] != 0, n, a);
}

// a = 2a mod n for a < n.
template <int NL>
__device__ __forceinline__ void mod_dbl(uint32_t (&a)[NL], const uint32_t (&n)[NL]) {
  const uint32_t top = a[NL - 1] >> 31;
#pragma unroll
  for (int j = NL - 1; j > 0; --j) a[j] = (a[j] << 1) | (a[j - 1] >> 31);
  a[0] <<= 1;
  sub_if_ge<NL>(a, top != 0, n, a);
}

// x * R^-1 mod n (Montgomery reduction) for x < n.
template <int NL>
__device__ __forceinline__ void mont_redc(const uint32_t (&x)[NL], const uint32_t (&n)[NL], uint32_t ninv,
                                          uint32_t (&y)[NL]) {
  uint32_t t[NL + 1];
#pragma unroll
  for (int j = 0; j < NL; ++j) t[j] = x[j];
  t[NL] = 0;
#pragma unroll 1
  for (int i = 0; i < NL; ++i) {
    const uint32_t q = t[0] * ninv;
    uint64_t s = (uint64_t)q * n[0] + t[0];
    uint32_t c = (uint32_t)(s >> 32);
#pragma unroll
    for (int j = 1; j < NL; ++j) {
      s = (uint64_t)q * n[j] + t[j] + c;
      t[j - 1] = (uint32_t)s;
      c = (uint32_t)(s >> 32);
    }
    s = (uint64_t)t[NL] + c;
    t[NL - 1] = (uint32_t)s;
    t[NL] = (uint32_t)(s >> 32);
  }
  sub_if_ge<NL>(t, t[NL] != 0, n, y);
}

// y == 1 / y == n - 1 (n odd).
template <int NL>
__device__ __forceinline__ bool is_one(const uint32_t (&y)[NL]) {
  uint32_t x = y[0] ^ 1u;
#pragma unroll
  for (int j = 1; j < NL; ++j) x |= y[j];
  return x == 0;
}
template <int NL>
__device__ __forceinline__ bool is_minus_one(const uint32_t (&y)[NL], const uint32_t (&n)[NL]) {
  uint32_t x = y[0] ^ (n[0] - 1u);
#pragma unroll
  for (int j = 1; j < NL; ++j) x |= y[j] ^ n[j];
  return x == 0;
}

// Limb i of n - 1 (n odd, so only limb 0 changes), i a runtime index.
template <int NL>
__device__ __forceinline__ uint32_t nm1_limb(const uint32_t (&n)[NL], int i) {
  uint32_t e = 0;
#pragma unroll
  for (int j = 0; j < NL; ++j) e = (j == i) ? n[j] : e;
  return i == 0 ? e - 1u : e;
}

// Strong probable-prime test to base 2 of n (any value below 2^(32 NL)).
template <int NL>
__device__ bool sprp2(const uint32_t (&n)[NL], uint32_t* __restrict__ b) {
  uint32_t hi = 0;
#pragma unroll
  for (int j = 1; j < NL; ++j) hi |= n[j];
  if (!(n[0] & 1u)) return hi == 0 && n[0] == 2u;
  if (hi == 0 && n[0] < 3u) return false;          // 1
  uint32_t inv = n[0];                              // n[0]^-1 mod 2^32 by Newton (3 -> 48 bits)
#pragma unroll
  for (int k = 0; k < 4; ++k) inv *= 2u - n[0] * inv;
  const uint32_t ninv = 0u - inv;
  int top = 0;
#pragma unroll
  for (int j = 0; j < NL; ++j) top = n[j] ? j : top;
  uint32_t ntop = 0;
#pragma unroll
  for (int j = 0; j < NL; ++j) ntop = (j == top) ? n[j] : ntop;
  const int bits = 32 * top + 32 - __clz(ntop);
  int s = 0;
  bool found = false;
#pragma unroll
  for (int j = 0; j < NL; ++j) {                    // n - 1 = 2^s t, t odd
    const uint32_t e = (j == 0) ? n[0] - 1u : n[j];
    if (!found && e) { s = 32 * j + __ffs(e) - 1; found = true; }
  }
  // x = 2R mod n (2 in Montgomery form): 2^(bits-1) < n doubled up to 2^(32 NL + 1)
  uint32_t x[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) x[j] = (j == ((bits - 1) >> 5)) ? (1u << ((bits - 1) & 31)) : 0u;
  for (int k = 0; k < 32 * NL - bits + 2; ++k) mod_dbl<NL>(x, n);
  // 2^t, left to right over the bits of t = bits [s, bits-1] of n - 1; the top bit (bits - 1)
  // is 1 and gave the starting value 2.
  uint32_t e = nm1_limb<NL>(n, (bits - 2) >> 5);
  for (int bit = bits - 2; bit >= s; --bit) {
    if ((bit & 31) == 31) e = nm1_limb<NL>(n, bit >> 5);
    mont_sqr<NL>(x, n, ninv, b);
    if ((e >> (bit & 31)) & 1u) mod_dbl<NL>(x, n);
  }
  uint32_t y[NL];
  mont_redc<NL>(x, n, ninv, y);
  if (is_one<NL>(y) || is_minus_one<NL>(y, n)) return true;
  for (int r = 1; r < s; ++r) {
    mont_sqr<NL>(x, n, ninv, b);
    mont_redc<NL>(x, n, ninv, y);
    if (is_minus_one<NL>(y, n)) return true;
    if (is_one<NL>(y)) return false;
  }
  return false;
}

// ---------------------------------------------------------------------------------------------
// The same test with a candidate spread over a quad of lanes, for NL = 4L limbs (L >= 3).  Lane r
// of a quad holds limbs [rL, rL + L) of each number, so a lane keeps three L-limb arrays (the
// value, the modulus and the accumulator) instead of three NL-limb ones: about a quarter of the
// registers, and four times the wavefronts per SIMD.  Limbs cross lanes by DPP quad permutations
// (a VALU operation, no LDS round trip).  Carries out of a lane's top limb are kept pending and
// enter the next lane at the next step, so no step waits for a carry to ripple through the quad;
// they are resolved once per squaring.  Every lane of a quad computes the same control values, so
// the quad stays converged.
// ---------------------------------------------------------------------------------------------
// DPP quad permutations: lane r of each quad reads lane SRC[r].
template <int SRC>
__device__ __forceinline__ uint32_t q_bcast(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, SRC * 0x55, 0xf, 0xf, false);          // (S, S, S, S)
}
__device__ __forceinline__ uint32_t q_from_prev(uint32_t v, uint32_t r) {    // lane r - 1 (lane 0: 0)
  const uint32_t x = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x90, 0xf, 0xf, false);   // (0, 0, 1, 2)
  return r ? x : 0u;
}
__device__ __forceinline__ uint32_t q_from_next(uint32_t v) {                 // lane r + 1 (lane 3: itself)
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xf9, 0xf, 0xf, false);               // (1, 2, 3, 3)
}
__device__ __forceinline__ uint32_t q_max(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xb1, 0xf, 0xf, false));          // (1, 0, 3, 2)
  return max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4e, 0xf, 0xf, false));       // (2, 3, 0, 1)
}
__device__ __forceinline__ uint32_t q_min(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xb1, 0xf, 0xf, false));
  return min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4e, 0xf, 0xf, false));
}
// every lane of the quad has the predicate (the quads of a wavefront are aligned to 4 lanes)
__device__ __forceinline__ bool q_all(bool p) {
  const unsigned long long b = __ballot(p);
  return ((b >> (__lane_id() & ~3u)) & 0xfull) == 0xfull;
}

// Carries pending out of each lane's top limb (pc, into the next lane's limb 0; lane 3's go to the
// word above the number, `top`) are added in; three rounds carry them across the quad.
template <int L>
__device__ __forceinline__ void q_resolve(uint32_t (&t)[L], uint32_t pc, uint32_t& top, uint32_t r) {
#pragma unroll
  for (int round = 0; round < 3; ++round) {
    uint32_t c = q_from_prev(pc, r);
    if (r == 3) top += pc;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const uint64_t s = (uint64_t)t[j] + c;
      t[j] = (uint32_t)s;
      c = (uint32_t)(s >> 32);
    }
    pc = c;
  }
  if (r == 3) top += pc;
}

// t = t - n if (top != 0 or t >= n), for a resolved t < 2n (top: the word above the number).
template <int L>
__device__ __forceinline__ void q_sub_if_ge(uint32_t (&t)[L], uint32_t top, const uint32_t (&n)[L], uint32_t r) {
  // this lane's borrow out of t - n for a borrow in of 0 (b0) and of 1 (b1 = b0 or t == n here)
  uint32_t br = 0, diff = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint64_t d = (uint64_t)t[j] - n[j] - br;
    br = (uint32_t)(d >> 32) & 1u;
    diff |= (uint32_t)d;
  }
  const uint32_t b0 = br, b1 = br | (diff == 0 ? 1u : 0u);
  uint32_t bin = 0;                                   // borrow into this lane, across the quad
#pragma unroll
  for (int round = 0; round < 3; ++round) bin = q_from_prev(bin ? b1 : b0, r);
  const uint32_t bout = bin ? b1 : b0;               // lane 3: borrow out of the whole t - n
  const bool sub = q_bcast<3>((top != 0 || bout == 0) ? 1u : 0u) != 0;
  if (!sub) return;
  br = bin;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint64_t d = (uint64_t)t[j] - n[j] - br;
    t[j] = (uint32_t)d;
    br = (uint32_t)(d >> 32) & 1u;
  }
}

// One row of the Montgomery product, t = t + x * y (y one limb), over this lane's limbs, with
// c_in entering limb 0; returns the carry out of the top limb.  Each limb of t sits in the low
// half of a 64-bit word whose high half stays 0, so x_j * y + t_j is one v_mad_u64_u32 that
// cannot overflow; the high halves of the products then go up one limb in a single
// add-with-carry chain.  SHIFT: the result is written one limb down (limb j + 1 into word j;
// limb 0 is returned through low0), which is the division by 2^32 of the reduction step.
template <int L, bool SHIFT>
__device__ __forceinline__ uint32_t q_row(uint64_t (&T)[L], const uint32_t (&x)[L], uint32_t y, uint32_t c_in,
                                          uint32_t* low0) {
  uint32_t prev = c_in, cy = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint64_t D = (uint64_t)x[j] * y + T[j];
    uint32_t co;
    const uint32_t v = __builtin_addc((uint32_t)D, prev, cy, &co);
    cy = co;
    prev = (uint32_t)(D >> 32);
    // (the high halves keep their zero register: only the low half is replaced)
    if (SHIFT) {
      if (j == 0) *low0 = v;
      else T[j - 1] = (T[j - 1] & 0xffffffff00000000ull) | v;
    } else {
      T[j] = (T[j] & 0xffffffff00000000ull) | v;
    }
  }
  return prev + cy;          // the lane's part of the sum fits in L + 1 limbs
}

// a = a*b/R mod n (R = 2^(32 NL)), a, b < n; col: this quad's LDS columns (lane o's limb l at
// col[l * kPrpBlock + o]), where b is written first so every lane can read the multiplier limbs.
template <int L>
__device__ __forceinline__ void q_mont_mul(uint32_t (&a)[L], const uint32_t (&b)[L], const uint32_t (&n)[L],
                                           uint32_t ninv, uint32_t r, uint32_t* own, const uint32_t* col) {
  // (own and col overlap: the writes must stay before the reads)
#pragma unroll
  for (int j = 0; j < L; ++j) own[j * kPrpBlock] = b[j];
  uint64_t T[L];
#pragma unroll
  for (int j = 0; j < L; ++j) T[j] = 0;
  uint32_t pc = 0, top = 0;
#pragma unroll 1
  for (int i = 0; i < 4 * L; ++i) {
    const int o = i / L, l = i - o * L;
    const uint32_t bi = col[l * kPrpBlock + o];      // limb i of the multiplier (owner lane o)
    // t += a * b_i, with the pending carry into this lane's limb 0
    const uint32_t ca = q_row<L, false>(T, a, bi, q_from_prev(pc, r), nullptr);
    const uint32_t q = q_bcast<0>((uint32_t)T[0] * ninv);   // lane 0's limb 0 is exact: t + q n = 0 mod 2^32
    // t = (t + q n) / 2^32: this lane's limbs move down one; lane r + 1's limb 0 (lane 3: the word
    // above) and this lane's pending carries become this lane's top limb
    uint32_t low0;
    const uint32_t c = q_row<L, true>(T, n, q, 0u, &low0);
    const uint32_t up = q_from_next(low0);
    const uint64_t h = (uint64_t)(r == 3 ? top : up) + ca + c;
    T[L - 1] = (T[L - 1] & 0xffffffff00000000ull) | (uint32_t)h;
    pc = (uint32_t)(h >> 32);
    if (r == 3) top = pc;
  }
  if (r == 3) pc = 0;                                 // lane 3's carry is `top` already
  uint32_t t[L];
#pragma unroll
  for (int j = 0; j < L; ++j) t[j] = (uint32_t)T[j];
  q_resolve<L>(t, pc, top, r);
  q_sub_if_ge<L>(t, top, n, r);
#pragma unroll
  for (int j = 0; j < L; ++j) a[j] = t[j];
}

// a = a*a/R mod n.
template <int L>
__device__ __forceinline__ void q_mont_sqr(uint32_t (&a)[L], const uint32_t (&n)[L], uint32_t ninv, uint32_t r,
                                           uint32_t* own, const uint32_t* col) {
  q_mont_mul<L>(a, a, n, ninv, r, own, col);
}

// a = 2a mod n for a < n.
template <int L>
__device__ __forceinline__ void q_mod_dbl(uint32_t (&a)[L], const uint32_t (&n)[L], uint32_t r) {
  const uint32_t hib = a[L - 1] >> 31;
  const uint32_t cin = q_from_prev(hib, r);
#pragma unroll
  for (int j = L - 1; j > 0; --j) a[j] = (a[j] << 1) | (a[j - 1] >> 31);
  a[0] = (a[0] << 1) | cin;
  q_sub_if_ge<L>(a, q_bcast<3>(hib), n, r);
}

// y = x R^-1 mod n (Montgomery reduction) for x < n.
template <int L>
__device__ __forceinline__ void q_mont_redc(const uint32_t (&x)[L], const uint32_t (&n)[L], uint32_t ninv,
                                            uint32_t r, uint32_t (&y)[L]) {
  uint32_t t[L];
#pragma unroll
  for (int j = 0; j < L; ++j) t[j] = x[j];
  uint32_t pc = 0, top = 0;
#pragma unroll 1
  for (int i = 0; i < 4 * L; ++i) {
    uint32_t c = q_from_prev(pc, r);
    const uint32_t q = q_bcast<0>((t[0] + c) * ninv);   // lane 0: c = 0
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const uint64_t s = (uint64_t)q * n[j] + t[j] + c;
      t[j] = (uint32_t)s;
      c = (uint32_t)(s >> 32);
    }
    const uint32_t up = q_from_next(t[0]);
#pragma unroll
    for (int j = 0; j < L - 1; ++j) t[j] = t[j + 1];
    const uint64_t h = (uint64_t)(r == 3 ? top : up) + c;
    t[L - 1] = (uint32_t)h;
    pc = (uint32_t)(h >> 32);
    if (r == 3) top = pc;
  }
  if (r == 3) pc = 0;
  q_resolve<L>(t, pc, top, r);
  q_sub_if_ge<L>(t, top, n, r);
#pragma unroll
  for (int j = 0; j < L; ++j) y[j] = t[j];
}

// Strong probable-prime test to base 2 of n (NL = 4L limbs spread over the quad); own/col: this
// lane's LDS column and the quad's (2L words per lane: the multiplier, then n).
template <int L>
__device__ bool q_sprp2(const uint32_t (&n)[L], uint32_t r, uint32_t* own, const uint32_t* col) {
  // the quad's n in LDS for the exponent bits
#pragma unroll
  for (int j = 0; j < L; ++j) own[(L + j) * kPrpBlock] = n[j];
  uint32_t hi_local = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) hi_local |= (r == 0 && j == 0) ? 0u : n[j];
  const bool hi_zero = q_all(hi_local == 0);
  const uint32_t n0 = q_bcast<0>(n[0]);
  if (!(n0 & 1u)) return hi_zero && n0 == 2u;
  if (hi_zero && n0 < 3u) return false;             // 1
  uint32_t inv = n0;                                 // n0^-1 mod 2^32 by Newton (3 -> 48 bits)
#pragma unroll
  for (int k = 0; k < 4; ++k) inv *= 2u - n0 * inv;
  const uint32_t ninv = 0u - inv;
  // bit length of n, and s with n - 1 = 2^s t, t odd
  uint32_t bl = 0, tz = 0xffffffffu;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint32_t g = r * L + j;
    if (n[j]) bl = 32 * g + 32 - __clz(n[j]);
    const uint32_t e = (r == 0 && j == 0) ? n[j] - 1u : n[j];
    if (e && tz == 0xffffffffu) tz = 32 * g + __ffs(e) - 1;
  }
  const int bits = (int)q_max(bl);
  const int s = (int)q_min(tz);
  auto nm1_limb = [&](int g) -> uint32_t {           // limb g of n - 1, from the quad's LDS copy
    const int o = g / L, l = g - o * L;
    const uint32_t v = col[(L + l) * kPrpBlock + o];
    return g == 0 ? v - 1u : v;
  };
  // x = 2R mod n: 2^(bits-1) < n doubled up to 2^(32 NL + 1)
  uint32_t x[L];
#pragma unroll
  for (int j = 0; j < L; ++j) x[j] = ((int)(r * L + j) == ((bits - 1) >> 5)) ? (1u << ((bits - 1) & 31)) : 0u;
  for (int k = 0; k < 32 * 4 * L - bits + 2; ++k) q_mod_dbl<L>(x, n, r);
  uint32_t e = nm1_limb((bits - 2) >> 5);
  for (int bit = bits - 2; bit >= s; --bit) {
    if ((bit & 31) == 31) e = nm1_limb(bit >> 5);
    q_mont_sqr<L>(x, n, ninv, r, own, col);
    if ((e >> (bit & 31)) & 1u) q_mod_dbl<L>(x, n, r);
  }
  uint32_t y[L];
  q_mont_redc<L>(x, n, ninv, r, y);
  auto is_one = [&]() {
    uint32_t d = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) d |= y[j] ^ ((r == 0 && j == 0) ? 1u : 0u);
    return q_all(d == 0);
  };
  auto is_minus_one = [&]() {
    uint32_t d = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) d |= y[j] ^ ((r == 0 && j == 0) ? n[j] - 1u : n[j]);
    return q_all(d == 0);
  };
  if (is_one() || is_minus_one()) return true;
  for (int k = 1; k < s; ++k) {
    q_mont_sqr<L>(x, n, ninv, r, own, col);
    q_mont_redc<L>(x, n, ninv, r, y);
    if (is_minus_one()) return true;
    if (is_one()) return false;
  }
  return false;
}

// ---------------------------------------------------------------------------------------------
// Strong Lucas test on a quad of lanes (the second half of BPSW).  Section 2.2: the search tests
// with GMP's probable-prime routine, a BPSW test.  Parameters after Selfridge: D the first of 5,
// -7, 9, -11, ... with Jacobi symbol (D/n) = -1, P = 1, Q = (1 - D)/4; with n + 1 = 2^s d, d odd,
// n passes iff U_d = 0 or V_(2^r d) = 0 (mod n) for some 0 <= r < s.  U, V and Q^k run in
// Montgomery form through the doubling formulas U_2k = U_k V_k, V_2k = V_k^2 - 2Q^k and the step
// U_(k+1) = (U_k + V_k)/2, V_(k+1) = (D U_k + V_k)/2, whose products by D and Q (small integers)
// are chains of doublings and additions.
// ---------------------------------------------------------------------------------------------
// Searched values of |D|: a non-square n has (D/n) = -1 for some |D| below 2 (ln n)^2 under the
// generalised Riemann hypothesis (4.1e6 for n < 2^2048); a search that reaches the bound reports
// n composite, which a perfect square (for which no such D exists) is.
constexpr uint32_t kLucasDMax = 1u << 23;

// Sum of a quad-uniform reduction: every lane gets v0 + v1 + v2 + v3 of its quad.
__device__ __forceinline__ uint64_t q_sum64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  uint64_t x = ((uint64_t)(uint32_t)__builtin_amdgcn_mov_dpp((int)hi, 0xb1, 0xf, 0xf, false) << 32) |
               (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, 0xb1, 0xf, 0xf, false);     // (1, 0, 3, 2)
  v += x;
  lo = (uint32_t)v;
  hi = (uint32_t)(v >> 32);
  x = ((uint64_t)(uint32_t)__builtin_amdgcn_mov_dpp((int)hi, 0x4e, 0xf, 0xf, false) << 32) |
      (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, 0x4e, 0xf, 0xf, false);              // (2, 3, 0, 1)
  return v + x;
}

// n mod q for 2 < q < 2^32 (q odd), n spread over the quad.
template <int L>
__device__ __forceinline__ uint32_t q_mod_u32(const uint32_t (&n)[L], uint32_t q, uint32_t r) {
  const uint64_t b = (uint64_t)(((uint64_t)1 << 32) % q);    // 2^32 mod q
  uint64_t w = 1;                                             // 2^(32 g) mod q for this lane's first limb
  for (uint32_t g = 0; g < r * L; ++g) w = w * b % q;
  uint64_t acc = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    acc = (acc + (uint64_t)(n[j] % q) * w) % q;
    w = w * b % q;
  }
  return (uint32_t)(q_sum64(acc) % q);
}

// Jacobi symbol (a/m) for odd m > 0, a < m (quadratic reciprocity and the rule for (2/m)).
__device__ __forceinline__ int jacobi_u32(uint32_t a, uint32_t m) {
  int t = 1;
  while (a != 0) {
    while ((a & 1u) == 0) {
      a >>= 1;
      const uint32_t m8 = m & 7u;
      if (m8 == 3 || m8 == 5) t = -t;
    }
    const uint32_t tmp = a;
    a = m;
    m = tmp;
    if ((a & 3u) == 3 && (m & 3u) == 3) t = -t;
    a %= m;
  }
  return m == 1 ? t : 0;
}

// t = a + b mod n for a, b < n.
template <int L>
__device__ __forceinline__ void q_mod_add(uint32_t (&t)[L], const uint32_t (&a)[L], const uint32_t (&b)[L],
                                          const uint32_t (&n)[L], uint32_t r) {
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint64_t v = (uint64_t)a[j] + b[j] + c;
    t[j] = (uint32_t)v;
    c = (uint32_t)(v >> 32);
  }
  uint32_t top = 0;
  q_resolve<L>(t, c, top, r);
  q_sub_if_ge<L>(t, top, n, r);
}

// t = a - b mod n for a, b < n: a + (2^(32 NL) - b), then n added back if that did not carry out.
template <int L>
__device__ __forceinline__ void q_mod_sub(uint32_t (&t)[L], const uint32_t (&a)[L], const uint32_t (&b)[L],
                                          const uint32_t (&n)[L], uint32_t r) {
  uint32_t c = r == 0 ? 1u : 0u;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint64_t v = (uint64_t)a[j] + (uint32_t)~b[j] + c;
    t[j] = (uint32_t)v;
    c = (uint32_t)(v >> 32);
  }
  uint32_t top = 0;
  q_resolve<L>(t, c, top, r);
  if (q_bcast<3>(top) != 0) return;                   // a >= b
  c = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint64_t v = (uint64_t)t[j] + n[j] + c;
    t[j] = (uint32_t)v;
    c = (uint32_t)(v >> 32);
  }
  uint32_t drop = 0;                                  // the carry out of 2^(32 NL)
  q_resolve<L>(t, c, drop, r);
}

// a = a / 2 mod n for a < n, n odd: (a + n) / 2 when a is odd.
template <int L>
__device__ __forceinline__ void q_half(uint32_t (&a)[L], const uint32_t (&n)[L], uint32_t r) {
  uint32_t top = 0;
  if (q_bcast<0>(a[0]) & 1u) {
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const uint64_t v = (uint64_t)a[j] + n[j] + c;
      a[j] = (uint32_t)v;
      c = (uint32_t)(v >> 32);
    }
    q_resolve<L>(a, c, top, r);
  }
  const uint32_t next_low = q_from_next(a[0]);        // lane r + 1's limb 0 (lane 3: the carry word)
  const uint32_t in_bit = (r == 3 ? top : next_low) & 1u;
#pragma unroll
  for (int j = 0; j < L - 1; ++j) a[j] = (a[j] >> 1) | (a[j + 1] << 31);
  a[L - 1] = (a[L - 1] >> 1) | (in_bit << 31);
}

template <int L>
__device__ __forceinline__ bool q_is_zero(const uint32_t (&a)[L]) {
  uint32_t d = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) d |= a[j];
  return q_all(d == 0);
}

// c R mod n for a small signed c, from one = R mod n by doubling and adding.
template <int L>
__device__ __forceinline__ void q_mont_small(uint32_t (&t)[L], int32_t c, const uint32_t (&one)[L],
                                             const uint32_t (&n)[L], uint32_t r) {
  const uint32_t a = (uint32_t)(c < 0 ? -c : c);
#pragma unroll
  for (int j = 0; j < L; ++j) t[j] = 0;
  for (int bit = 31 - __clz(a); bit >= 0; --bit) {
    q_mod_dbl<L>(t, n, r);
    if ((a >> bit) & 1u) q_mod_add<L>(t, t, one, n, r);
  }
  if (c < 0) {
    uint32_t z[L];
#pragma unroll
    for (int j = 0; j < L; ++j) z[j] = 0;
    q_mod_sub<L>(t, z, t, n, r);
  }
}

// t = c x mod n for a small signed c != 0 and x < n (any form: the product of a residue in
// Montgomery form by an integer stays in that form), by doubling and adding; t may alias x.
template <int L>
__device__ __forceinline__ void q_mul_small(uint32_t (&t)[L], const uint32_t (&x)[L], int32_t c,
                                            const uint32_t (&n)[L], uint32_t r) {
  const uint32_t a = (uint32_t)(c < 0 ? -c : c);
  uint32_t y[L], acc[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    y[j] = x[j];
    acc[j] = x[j];                                             // the top bit of a
  }
  for (int bit = 30 - __clz(a); bit >= 0; --bit) {
    q_mod_dbl<L>(acc, n, r);
    if ((a >> bit) & 1u) q_mod_add<L>(acc, acc, y, n, r);
  }
  if (c < 0) {
    uint32_t z[L];
#pragma unroll
    for (int j = 0; j < L; ++j) z[j] = 0;
    q_mod_sub<L>(acc, z, acc, n, r);
  }
#pragma unroll
  for (int j = 0; j < L; ++j) t[j] = acc[j];
}

// Strong Lucas probable-prime test of n (NL = 4L limbs spread over the quad); own/col as in
// q_sprp2 (the second L words of each lane's column receive n + 1).
template <int L>
__device__ bool q_strong_lucas(const uint32_t (&n)[L], uint32_t r, uint32_t* own, const uint32_t* col) {
  uint32_t hi_local = 0, ones = 0xffffffffu;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    hi_local |= (r == 0 && j == 0) ? 0u : n[j];
    ones &= n[j];
  }
  const bool hi_zero = q_all(hi_local == 0);
  const uint32_t n0 = q_bcast<0>(n[0]);
  if (!(n0 & 1u)) return hi_zero && n0 == 2u;
  if (hi_zero && n0 < 3u) return false;               // 1
  if (q_all(ones == 0xffffffffu)) return false;       // 2^(32 NL) - 1: composite (32 NL is even)
  if (hi_zero) {                                      // a square below 2^32 has no D below
    const uint32_t s0 = (uint32_t)sqrt((double)n0);
    for (uint32_t x = s0 > 0 ? s0 - 1 : 0; x <= s0 + 1; ++x)
      if ((uint64_t)x * x == n0) return false;
  }
  // D: the first of 5, -7, 9, -11, ... with (D/n) = -1
  int32_t D = 5;
  for (;;) {
    const uint32_t q = (uint32_t)(D < 0 ? -D : D);
    const uint32_t nm = q_mod_u32<L>(n, q, r);
    int j = jacobi_u32(nm, q);
    if (j == 0) {
      if (!(hi_zero && n0 == q)) return false;        // 1 < gcd(q, n) <= q < n: n is composite
    } else {
      // (|D|/n) = (n/|D|) (-1)^((|D|-1)/2 (n-1)/2); (-1/n) = (-1)^((n-1)/2)
      if ((q & 3u) == 3 && (n0 & 3u) == 3) j = -j;
      if (D < 0 && (n0 & 3u) == 3) j = -j;
      if (j == -1) break;
    }
    if (q >= kLucasDMax) return false;
    D = D > 0 ? -(D + 2) : -D + 2;
  }
  const int32_t Q = (1 - D) / 4;
  // n + 1, kept in LDS for its bits; s = its trailing zeros, bl = its bit length
  uint32_t np1[L];
  {
    uint32_t c = r == 0 ? 1u : 0u;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const uint64_t v = (uint64_t)n[j] + c;
      np1[j] = (uint32_t)v;
      c = (uint32_t)(v >> 32);
    }
    uint32_t top = 0;
    q_resolve<L>(np1, c, top, r);                    // no carry out: n is not 2^(32 NL) - 1
  }
#pragma unroll
  for (int j = 0; j < L; ++j) own[(L + j) * kPrpBlock] = np1[j];
  uint32_t bl = 0, tz = 0xffffffffu;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint32_t g = r * L + j;
    if (np1[j]) bl = 32 * g + 32 - __clz(np1[j]);
    if (np1[j] && tz == 0xffffffffu) tz = 32 * g + __ffs(np1[j]) - 1;
  }
  const int bits = (int)q_max(bl);
  const int s = (int)q_min(tz);
  auto np1_bit = [&](int bit) -> uint32_t {
    const int g = bit >> 5, o = g / L, l = g - o * L;
    return (col[(L + l) * kPrpBlock + o] >> (bit & 31)) & 1u;
  };
  // Montgomery constants: ninv = -n^-1 mod 2^32; one = R mod n from the largest power of two below n
  uint32_t inv = n0;
#pragma unroll
  for (int k = 0; k < 4; ++k) inv *= 2u - n0 * inv;
  const uint32_t ninv = 0u - inv;
  uint32_t nbl = 0;
#pragma unroll
  for (int j = 0; j < L; ++j)
    if (n[j]) nbl = 32 * (r * L + j) + 32 - __clz(n[j]);
  const int nbits = (int)q_max(nbl);
  uint32_t one[L];
#pragma unroll
  for (int j = 0; j < L; ++j) one[j] = ((int)(r * L + j) == ((nbits - 1) >> 5)) ? (1u << ((nbits - 1) & 31)) : 0u;
  for (int k = 0; k < 32 * 4 * L - nbits + 1; ++k) q_mod_dbl<L>(one, n, r);
  uint32_t Qm[L];
  q_mont_small<L>(Qm, Q, one, n, r);
  // U_1 = 1, V_1 = P = 1, Q^1; then the bits of d = (n + 1) / 2^s below its top bit
  uint32_t U[L], V[L], Qk[L], t[L], w[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    U[j] = one[j];
    V[j] = one[j];
    Qk[j] = Qm[j];
  }
  for (int bit = bits - 2; bit >= s; --bit) {
    q_mont_mul<L>(U, V, n, ninv, r, own, col);                        // U_2k = U_k V_k
    q_mont_sqr<L>(V, n, ninv, r, own, col);
    q_mod_add<L>(t, Qk, Qk, n, r);
    q_mod_sub<L>(V, V, t, n, r);                                      // V_2k = V_k^2 - 2 Q^k
    q_mont_sqr<L>(Qk, n, ninv, r, own, col);                          // Q^2k
    if (np1_bit(bit)) {
      q_mul_small<L>(w, U, D, n, r);                                  // D U_k (|D| small)
      q_mod_add<L>(t, U, V, n, r);
      q_half<L>(t, n, r);                                             // U_(k+1) = (U_k + V_k) / 2
      q_mod_add<L>(w, w, V, n, r);
      q_half<L>(w, n, r);                                             // V_(k+1) = (D U_k + V_k) / 2
#pragma unroll
      for (int j = 0; j < L; ++j) {
        U[j] = t[j];
        V[j] = w[j];
      }
      q_mul_small<L>(Qk, Qk, Q, n, r);                                // Q^(k+1) (|Q| small)
    }
  }
  if (q_is_zero<L>(U) || q_is_zero<L>(V)) return true;
  for (int k = 1; k < s; ++k) {
    q_mont_sqr<L>(V, n, ninv, r, own, col);
    q_mod_add<L>(t, Qk, Qk, n, r);
    q_mod_sub<L>(V, V, t, n, r);                                      // V_(2^k d)
    if (q_is_zero<L>(V)) return true;
    q_mont_sqr<L>(Qk, n, ninv, r, own, col);
  }
  return false;
}

// Any of the tests on numbers given as limbs (a quad of lanes per number): test = CS_PRP_SPRP2,
// CS_PRP_LUCAS or CS_PRP_BPSW (both, the Lucas test only for numbers passing the first).
template <int L>
__global__ __launch_bounds__(kPrpBlock) void k_prp_test_q(const uint32_t* __restrict__ limbs, uint32_t n_limbs,
                                                          uint64_t count, uint32_t test, uint8_t* __restrict__ out) {
  extern __shared__ uint32_t lds[];
  const uint64_t i = (blockIdx.x * (uint64_t)kPrpBlock + threadIdx.x) / 4;
  if (i >= count) return;                            // whole quads leave together
  const uint32_t r = threadIdx.x & 3u;
  uint32_t v[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint32_t g = r * L + j;
    v[j] = g < n_limbs ? limbs[i * n_limbs + g] : 0u;
  }
  bool pp = true;
  if (test != CS_PRP_LUCAS) pp = q_sprp2<L>(v, r, lds + threadIdx.x, lds + (threadIdx.x & ~3u));
  if (pp && test != CS_PRP_SPRP2) pp = q_strong_lucas<L>(v, r, lds + threadIdx.x, lds + (threadIdx.x & ~3u));
  if (r == 0) out[i] = pp ? 1 : 0;
}

template <int L>
__global__ __launch_bounds__(kPrpBlock) void k_prp_numbers_q(const uint32_t* __restrict__ limbs, uint32_t n_limbs,
                                                             uint64_t count, uint8_t* __restrict__ out) {
  extern __shared__ uint32_t lds[];
  const uint64_t i = (blockIdx.x * (uint64_t)kPrpBlock + threadIdx.x) / 4;
  if (i >= count) return;                            // whole quads leave together
  const uint32_t r = threadIdx.x & 3u;
  uint32_t v[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint32_t g = r * L + j;
    v[j] = g < n_limbs ? limbs[i * n_limbs + g] : 0u;
  }
  const bool pp = q_sprp2<L>(v, r, lds + threadIdx.x, lds + (threadIdx.x & ~3u));
  if (r == 0) out[i] = pp ? 1 : 0;
}

template <int NL>
__global__ __launch_bounds__(kPrpBlock) void k_prp_numbers(const uint32_t* __restrict__ limbs, uint32_t n_limbs,
                                                           uint64_t count, uint8_t* __restrict__ out) {
  extern __shared__ uint32_t lds[];
  const uint64_t i = blockIdx.x * (uint64_t)kPrpBlock + threadIdx.x;
  if (i >= count) return;
  uint32_t v[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) v[j] = (uint32_t)j < n_limbs ? limbs[i * n_limbs + j] : 0u;
  out[i] = sprp2<NL>(v, lds + threadIdx.x) ? 1 : 0;
}

// ---------------------------------------------------------------------------------------------
// Surrounding primes.  A task is one side of one row: task = 2 row + side (side 0 walks down from
// the largest negative column, side 1 up from the smallest positive one).  Each round gathers the
// next B unmarked columns of every open task, tests them all, and closes the tasks whose batch
// holds a probable prime (the first one in walking order) or that ran out of columns.
// ---------------------------------------------------------------------------------------------
struct SurroundDev {
  const uint32_t* bitmap;     // n_rows x row_words, bit = 1: marked composite
  const uint64_t* m;          // m of each row
  const uint32_t* klimbs;     // K, NL limbs
  const int32_t* x_of_col;    // n_x
  int32_t* cur;               // per task: next column to look at
  int32_t* nxt;               // per task: where the current batch ended
  int32_t* slot_col;          // per slot: column, or -1
  uint8_t* slot_res;          // per slot: 1 if probable prime
  uint32_t* act[2];           // open-task lists (ping-pong)
  uint32_t* n_act;            // [0], [1] list sizes; [2] error flags
  unsigned long long* tests;  // [0] strong tests to base 2 run, [1] strong Lucas tests run
  cs_surround_row* out;
  uint64_t n_rows, m_lo, m_hi;
  uint32_t row_words, n_x;
  int32_t c_neg, c_pos;       // largest column with X < 0, smallest with X > 0 (-1 / n_x if none)
};

__global__ void k_sv_init(SurroundDev sv) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t >= 2 * sv.n_rows) return;
  sv.cur[t] = (t & 1) ? sv.c_pos : sv.c_neg;
  sv.act[0][t] = (uint32_t)t;
  if ((t & 1) == 0) {
    cs_surround_row z;
    z.prev = 0;
    z.next = 0;
    z.tests_prev = 0;
    z.tests_next = 0;
    sv.out[t >> 1] = z;
  }
}

// Up to B unmarked columns of each open task, in walking order, into slots [i B, i B + B).
__global__ void k_sv_gather(SurroundDev sv, uint32_t in, uint32_t n_open, uint32_t B) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_open) return;
  const uint32_t task = sv.act[in][i];
  const uint64_t row = task >> 1;
  const uint32_t* __restrict__ w = sv.bitmap + row * sv.row_words;
  int32_t* __restrict__ slots = sv.slot_col + (uint64_t)i * B;
  int32_t c = sv.cur[task];
  uint32_t k = 0;
  if (task & 1) {                                   // upwards to n_x - 1
    while (k < B && c < (int32_t)sv.n_x) {
      const int32_t wbase = c & ~31;
      uint32_t free_bits = ~w[c >> 5] & (0xffffffffu << (c & 31));
      while (free_bits && k < B) {
        const int32_t col = wbase + __ffs(free_bits) - 1;
        if (col >= (int32_t)sv.n_x) { free_bits = 0; break; }   // padding bits of the last word
        slots[k++] = col;
        free_bits &= free_bits - 1;
        c = col + 1;
      }
      if (k < B) c = wbase + 32;                    // this word has no free column left
    }
  } else {                                          // downwards to 0
    while (k < B && c >= 0) {
      const int32_t wbase = c & ~31;
      uint32_t free_bits = ~w[c >> 5] & (0xffffffffu >> (31 - (c & 31)));
      while (free_bits && k < B) {
        const int32_t col = wbase + 31 - __clz(free_bits);
        slots[k++] = col;
        free_bits &= ~(1u << (col & 31));
        c = col - 1;
      }
      if (k < B) c = wbase - 1;
    }
  }
  sv.nxt[task] = c;
  for (uint32_t r = k; r < B; ++r) slots[r] = -1;
}

template <int NL>
__global__ __launch_bounds__(kPrpBlock) void k_sv_test(SurroundDev sv, uint32_t in, uint64_t n_slots, uint32_t B) {
  extern __shared__ uint32_t lds[];
  const uint64_t sidx = blockIdx.x * (uint64_t)kPrpBlock + threadIdx.x;
  if (sidx >= n_slots) return;
  const int32_t col = sv.slot_col[sidx];
  const unsigned long long live = __ballot(col >= 0);
  if ((threadIdx.x & (kWave - 1)) == 0 && live) atomicAdd(sv.tests, (unsigned long long)__popcll(live));
  if (col < 0) {
    sv.slot_res[sidx] = 0;
    return;
  }
  const uint32_t task = sv.act[in][sidx / B];
  const uint64_t m = sv.m[task >> 1];
  if (m < sv.m_lo || m >= sv.m_hi) {                // outside the job's range: no result
    atomicOr(&sv.n_act[2], 1u);
    sv.slot_res[sidx] = 0;
    return;
  }
  const int32_t X = sv.x_of_col[col];
  // N = m K + X
  uint32_t v[NL];
  const uint32_t mlo = (uint32_t)m, mhi = (uint32_t)(m >> 32);
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const uint64_t s = (uint64_t)sv.klimbs[j] * mlo + c;
    v[j] = (uint32_t)s;
    c = (uint32_t)(s >> 32);
  }
  if (mhi) {
    c = 0;
#pragma unroll
    for (int j = 1; j < NL; ++j) {
      const uint64_t s = (uint64_t)sv.klimbs[j - 1] * mhi + v[j] + c;
      v[j] = (uint32_t)s;
      c = (uint32_t)(s >> 32);
    }
  }
  if (X >= 0) {
    uint32_t cy = (uint32_t)X;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const uint64_t s = (uint64_t)v[j] + cy;
      v[j] = (uint32_t)s;
      cy = (uint32_t)(s >> 32);
    }
  } else {
    uint32_t bw = (uint32_t)(-X);
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const uint64_t s = (uint64_t)v[j] - bw;
      v[j] = (uint32_t)s;
      bw = (uint32_t)(s >> 32) & 1u;
    }
  }
  sv.slot_res[sidx] = sprp2<NL>(v, lds + threadIdx.x) ? 1 : 0;
}

// N = m K + X on a quad of lanes (K has kl limbs, at most 4L): each lane forms its limbs, the
// carries out of its top limb resolved across the quad after each pass (N < 2^(32 NL), so nothing
// leaves the quad).
template <int L>
__device__ __forceinline__ void q_sv_number(const SurroundDev& sv, uint32_t kl, uint64_t m, int32_t X, uint32_t r,
                                            uint32_t (&v)[L]) {
  uint32_t dummy = 0;
  const uint32_t mlo = (uint32_t)m, mhi = (uint32_t)(m >> 32);
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint32_t g = r * L + j;
    const uint64_t s = (uint64_t)(g < kl ? sv.klimbs[g] : 0u) * mlo + c;
    v[j] = (uint32_t)s;
    c = (uint32_t)(s >> 32);
  }
  q_resolve<L>(v, c, dummy, r);
  if (mhi) {                                          // the same quad-uniform branch in every lane
    c = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const uint32_t g = r * L + j;
      const uint64_t s = (uint64_t)(g && g - 1 < kl ? sv.klimbs[g - 1] : 0u) * mhi + v[j] + c;
      v[j] = (uint32_t)s;
      c = (uint32_t)(s >> 32);
    }
    q_resolve<L>(v, c, dummy, r);
  }
  // + X, or + (2^(32 NL) - |X|) with the carry out of the number dropped
  const bool neg = X < 0;
  const uint32_t ax = (uint32_t)(neg ? -X : X);
  c = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const bool low = r == 0 && j == 0;
    const uint32_t add = neg ? (low ? 0u - ax : 0xffffffffu) : (low ? ax : 0u);
    const uint64_t s = (uint64_t)v[j] + add + c;
    v[j] = (uint32_t)s;
    c = (uint32_t)(s >> 32);
  }
  q_resolve<L>(v, c, dummy, r);
}

// The same on a quad of lanes per candidate (NL = 4L limbs).
// Wavefronts per SIMD the register allocation of k_sv_test_q aims for: at 10 to 12 limbs per
// lane (numbers of 1,280 to 1,536 bits) the squaring loop fits in 96 VGPRs without spills (only a
// few values of the per-squaring carry resolution go to scratch), for five wavefronts instead of
// four; elsewhere the compiler's own choice.
template <int L>
constexpr int sv_min_waves() { return (L >= 10 && L <= 12) ? 5 : 1; }

template <int L>
__global__ __launch_bounds__(kPrpBlock) __attribute__((amdgpu_waves_per_eu(sv_min_waves<L>())))
void k_sv_test_q(SurroundDev sv, uint32_t in, uint64_t n_slots, uint32_t B) {
  extern __shared__ uint32_t lds[];
  const uint64_t sidx = (blockIdx.x * (uint64_t)kPrpBlock + threadIdx.x) / 4;
  if (sidx >= n_slots) return;                       // whole quads leave together
  const uint32_t r = threadIdx.x & 3u;
  const int32_t col = sv.slot_col[sidx];
  const unsigned long long live = __ballot(col >= 0 && r == 0);
  if ((threadIdx.x & (kWave - 1)) == 0 && live) atomicAdd(sv.tests, (unsigned long long)__popcll(live));
  if (col < 0) {
    if (r == 0) sv.slot_res[sidx] = 0;
    return;
  }
  const uint32_t task = sv.act[in][sidx / B];
  const uint64_t m = sv.m[task >> 1];
  if (m < sv.m_lo || m >= sv.m_hi) {                // outside the job's range: no result
    if (r == 0) {
      atomicOr(&sv.n_act[2], 1u);
      sv.slot_res[sidx] = 0;
    }
    return;
  }
  const int32_t X = sv.x_of_col[col];
  uint32_t v[L];
  q_sv_number<L>(sv, 4 * L, m, X, r, v);
  const bool pp = q_sprp2<L>(v, r, lds + threadIdx.x, lds + (threadIdx.x & ~3u));
  if (r == 0) sv.slot_res[sidx] = pp ? 1 : 0;
}

__global__ void k_sv_resolve(SurroundDev sv, uint32_t in, uint32_t n_open, uint32_t B) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_open) return;
  const uint32_t task = sv.act[in][i];
  const uint64_t row = task >> 1;
  const uint64_t base = (uint64_t)i * B;
  uint32_t k = 0;
  int32_t hit = 0;
  bool closed = false;
  for (; k < B; ++k) {
    const int32_t col = sv.slot_col[base + k];
    if (col < 0) { closed = true; break; }          // no columns left on this side
    if (sv.slot_res[base + k]) { hit = sv.x_of_col[col]; ++k; closed = true; break; }
  }
  cs_surround_row& o = sv.out[row];
  if (task & 1) o.tests_next += k;
  else o.tests_prev += k;
  if (closed) {
    if (task & 1) o.next = hit;
    else o.prev = hit;
  } else {
    sv.cur[task] = sv.nxt[task];
    const uint32_t at = atomicAdd(&sv.n_act[in ^ 1], 1u);
    sv.act[in ^ 1][at] = task;
  }
}

// The second half of BPSW for every side's probable prime (sides with none are skipped): the
// strong Lucas test of N + X on a quad of lanes (K has kl limbs).  A side whose number fails (a
// strong pseudoprime to base 2) is reopened just past it and appended to list `fail`.
template <int L>
__global__ __launch_bounds__(kPrpBlock) void k_sv_lucas_q(SurroundDev sv, uint32_t kl, uint32_t fail, uint64_t n_tasks) {
  extern __shared__ uint32_t lds[];
  const uint64_t task = (blockIdx.x * (uint64_t)kPrpBlock + threadIdx.x) / 4;
  if (task >= n_tasks) return;                        // whole quads leave together
  const uint32_t r = threadIdx.x & 3u;
  const uint64_t row = task >> 1;
  cs_surround_row& o = sv.out[row];
  const int32_t X = (task & 1) ? o.next : o.prev;
  if (X == 0) return;                                 // no probable prime on this side
  if (r == 0) atomicAdd(sv.tests + 1, 1ull);
  uint32_t v[L];
  q_sv_number<L>(sv, kl, sv.m[row], X, r, v);
  if (q_strong_lucas<L>(v, r, lds + threadIdx.x, lds + (threadIdx.x & ~3u)) || r != 0) return;
  // its column (x_of_col ascends), and the search resumes at the next one in walking order
  uint32_t lo = 0, hi = sv.n_x;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (sv.x_of_col[mid] <= X) lo = mid;
    else hi = mid;
  }
  if (task & 1) o.next = 0;
  else o.prev = 0;
  sv.cur[task] = (task & 1) ? (int32_t)lo + 1 : (int32_t)lo - 1;
  const uint32_t at = atomicAdd(&sv.n_act[fail], 1u);
  sv.act[fail][at] = (uint32_t)task;
}

// ------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------
#define PRP_INSTANCES(X) X(2) X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(36) X(40) X(44) X(48) X(52) X(56) X(60) X(64)

uint32_t pick_nl(uint32_t limbs) {
  static const uint32_t nls[] = {2, 4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48, 52, 56, 60, 64};
  for (uint32_t nl : nls)
    if (nl >= limbs) return nl;
  return 0;
}

// From 12 limbs a candidate takes a quad of lanes (L = NL / 4 limbs each, 2L LDS words per lane);
// below that one lane (NL LDS words per lane).
#define PRP_QUAD_INSTANCES(X) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
constexpr uint32_t kQuadMinNl = 12;

hipError_t launch_prp_numbers(uint32_t nl, const uint32_t* limbs, uint32_t n_limbs, uint64_t count, uint8_t* out,
                              hipStream_t s) {
  if (nl >= kQuadMinNl) {
    const uint32_t blocks = (uint32_t)((count * 4 + kPrpBlock - 1) / kPrpBlock);
    const size_t lds = (size_t)(nl / 2) * kPrpBlock * 4;
    switch (nl / 4) {
#define QCASE(L)                                                                                               \
  case L:                                                                                                      \
    hipLaunchKernelGGL(k_prp_numbers_q<L>, dim3(blocks), dim3(kPrpBlock), lds, s, limbs, n_limbs, count, out); \
    break;
      PRP_QUAD_INSTANCES(QCASE)
#undef QCASE
      default: return hipErrorInvalidValue;
    }
    return record_launch("k_prp_numbers_q");
  }
  const uint32_t blocks = (uint32_t)((count + kPrpBlock - 1) / kPrpBlock);
  const size_t lds = (size_t)nl * kPrpBlock * 4;
  switch (nl) {
#define CASE(N)                                                                                             \
  case N:                                                                                                   \
    hipLaunchKernelGGL(k_prp_numbers<N>, dim3(blocks), dim3(kPrpBlock), lds, s, limbs, n_limbs, count, out); \
    break;
    PRP_INSTANCES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return record_launch("k_prp_numbers");
}

// The strong Lucas or BPSW test on a quad of lanes per number, L = nl / 4 limbs per lane (at
// least 3).
hipError_t launch_prp_test(uint32_t nl, const uint32_t* limbs, uint32_t n_limbs, uint64_t count, uint32_t test,
                           uint8_t* out, hipStream_t s) {
  const uint32_t L = nl / 4 < 3 ? 3 : nl / 4;
  const uint32_t blocks = (uint32_t)((count * 4 + kPrpBlock - 1) / kPrpBlock);
  const size_t lds = (size_t)(2 * L) * kPrpBlock * 4;
  switch (L) {
#define TCASE(LL)                                                                                                  \
  case LL:                                                                                                         \
    hipLaunchKernelGGL(k_prp_test_q<LL>, dim3(blocks), dim3(kPrpBlock), lds, s, limbs, n_limbs, count, test, out); \
    break;
    PRP_QUAD_INSTANCES(TCASE)
#undef TCASE
    default: return hipErrorInvalidValue;
  }
  return record_launch("k_prp_test_q");
}

hipError_t launch_sv_lucas(uint32_t nl, const SurroundDev& sv, uint32_t kl, uint32_t fail, uint64_t n_tasks,
                           hipStream_t s) {
  const uint32_t L = nl / 4 < 3 ? 3 : nl / 4;
  const uint32_t blocks = (uint32_t)((n_tasks * 4 + kPrpBlock - 1) / kPrpBlock);
  const size_t lds = (size_t)(2 * L) * kPrpBlock * 4;
  switch (L) {
#define LCASE(LL)                                                                                            \
  case LL:                                                                                                   \
    hipLaunchKernelGGL(k_sv_lucas_q<LL>, dim3(blocks), dim3(kPrpBlock), lds, s, sv, kl, fail, n_tasks);      \
    break;
    PRP_QUAD_INSTANCES(LCASE)
#undef LCASE
    default: return hipErrorInvalidValue;
  }
  return record_launch("k_sv_lucas_q");
}

hipError_t launch_sv_test(uint32_t nl, const SurroundDev& sv, uint32_t in, uint64_t n_slots, uint32_t B,
                          hipStream_t s) {
  if (nl >= kQuadMinNl) {
    const uint32_t blocks = (uint32_t)((n_slots * 4 + kPrpBlock - 1) / kPrpBlock);
    const size_t lds = (size_t)(nl / 2) * kPrpBlock * 4;
    switch (nl / 4) {
#define QCASE(L)                                                                                     \
  case L:                                                                                            \
    hipLaunchKernelGGL(k_sv_test_q<L>, dim3(blocks), dim3(kPrpBlock), lds, s, sv, in, n_slots, B);   \
    break;
      PRP_QUAD_INSTANCES(QCASE)
#undef QCASE
      default: return hipErrorInvalidValue;
    }
    return record_launch("k_sv_test_q");
  }
  const uint32_t blocks = (uint32_t)((n_slots + kPrpBlock - 1) / kPrpBlock);
  const size_t lds = (size_t)nl * kPrpBlock * 4;
  switch (nl) {
#define CASE(N)                                                                                      \
  case N:                                                                                            \
    hipLaunchKernelGGL(k_sv_test<N>, dim3(blocks), dim3(kPrpBlock), lds, s, sv, in, n_slots, B);      \
    break;
    PRP_INSTANCES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return record_launch("k_sv_test");
}

// Candidates the test kernel of this limb count holds at once on the device (its occupancy by
// registers and LDS): a round of fewer candidates costs as much as a round of this many.
uint64_t sv_resident(uint32_t nl) {
  int per_cu = 0;
  hipError_t e = hipErrorInvalidValue;
  if (nl >= kQuadMinNl) {
    const size_t lds = (size_t)(nl / 2) * kPrpBlock * 4;
    switch (nl / 4) {
#define QOCC(L) \
  case L: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sv_test_q<L>, kPrpBlock, lds); break;
      PRP_QUAD_INSTANCES(QOCC)
#undef QOCC
      default: break;
    }
  } else {
    const size_t lds = (size_t)nl * kPrpBlock * 4;
    switch (nl) {
#define OCC(N) \
  case N: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sv_test<N>, kPrpBlock, lds); break;
      PRP_INSTANCES(OCC)
#undef OCC
      default: break;
    }
  }
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const uint64_t per_block = nl >= kQuadMinNl ? kPrpBlock / 4 : kPrpBlock;
  return (uint64_t)device_cu_count() * (uint64_t)per_cu * per_block;
}

// K = product of the primes dividing K, as 32-bit limbs (little endian).
std::vector<uint32_t> k_limbs(const std::vector<uint32_t>& kq) {
  std::vector<uint32_t> k(1, 1u);
  for (uint32_t q : kq) {
    uint64_t c = 0;
    for (auto& l : k) {
      const uint64_t s = (uint64_t)l * q + c;
      l = (uint32_t)s;
      c = s >> 32;
    }
    if (c) k.push_back((uint32_t)c);
  }
  return k;
}

uint32_t bit_length(const std::vector<uint32_t>& v) {
  for (size_t i = v.size(); i-- > 0;)
    if (v[i]) return (uint32_t)(32 * i + 32 - __builtin_clz(v[i]));
  return 0;
}

struct SvLayout {
  uint64_t klimbs, xcol, cur, nxt, act0, act1, n_act, slot_col, slot_res, total, slots;
};

SvLayout sv_layout(uint32_t nl, uint32_t n_x, uint64_t n_rows) {
  SvLayout L;
  uint64_t o = 0;
  auto take = [&](uint64_t b) { uint64_t at = o; o = (o + std::max<uint64_t>(b, 8) + 255) & ~255ull; return at; };
  const uint64_t tasks = 2 * n_rows;
  L.slots = std::max<uint64_t>(tasks * kSurroundB0, kSurroundSlotsMin);
  L.klimbs = take(nl * 4ull);
  L.xcol = take(n_x * 4ull);
  L.cur = take(tasks * 4);
  L.nxt = take(tasks * 4);
  L.act0 = take(tasks * 4);
  L.act1 = take(tasks * 4);
  L.n_act = take(32);
  L.slot_col = take(L.slots * 4);
  L.slot_res = take(L.slots);
  L.total = o;
  return L;
}

// Host description of a surround call: plan, K limbs, limb count.
cs_status surround_setup(const cs_job* job, Plan* pl, std::vector<uint32_t>* kl, uint32_t* nl) {
  cs_status st = make_plan(job, nullptr, 256, pl);
  if (st) return st;
  *kl = k_limbs(pl->kq);
  const uint64_t m_max = pl->job.m_start + pl->job.m_inc - 1;
  const uint32_t bits = bit_length(*kl) + (64 - __builtin_clzll(m_max)) + 1;   // m K + sl < 2^bits
  *nl = pick_nl((bits + 31) / 32);
  return *nl ? CS_OK : CS_ERANGE;
}

}  // namespace
}  // namespace cs

using namespace cs;

extern "C" cs_status cs_prp_numbers(const uint32_t* d_limbs, uint32_t n_limbs, uint64_t n, uint8_t* d_out,
                                    void* stream) {
  if (n == 0) return CS_OK;
  if (!d_limbs || !d_out || n_limbs == 0) return CS_EINVAL;
  const uint32_t nl = pick_nl(n_limbs);
  if (!nl) return CS_ERANGE;
  if (n > (1ull << 40)) return CS_ERANGE;
  return launch_prp_numbers(nl, d_limbs, n_limbs, n, d_out, static_cast<hipStream_t>(stream)) == hipSuccess
             ? CS_OK
             : CS_EDEVICE;
}

extern "C" cs_status cs_prp_test(const uint32_t* d_limbs, uint32_t n_limbs, uint64_t n, uint32_t test,
                                 uint8_t* d_out, void* stream) {
  if (test > CS_PRP_BPSW) return CS_EINVAL;
  if (test == CS_PRP_SPRP2) return cs_prp_numbers(d_limbs, n_limbs, n, d_out, stream);
  if (n == 0) return CS_OK;
  if (!d_limbs || !d_out || n_limbs == 0) return CS_EINVAL;
  const uint32_t nl = pick_nl(n_limbs);
  if (!nl) return CS_ERANGE;
  if (n > (1ull << 40)) return CS_ERANGE;
  return launch_prp_test(nl, d_limbs, n_limbs, n, test, d_out, static_cast<hipStream_t>(stream)) == hipSuccess
             ? CS_OK
             : CS_EDEVICE;
}

extern "C" cs_status cs_surround_ws(const cs_job* job, uint64_t n_rows, uint64_t* ws_bytes) {
  if (!job || !ws_bytes) return CS_EINVAL;
  if (n_rows >= (1ull << 30)) return CS_ERANGE;
  Plan pl;
  std::vector<uint32_t> kl;
  uint32_t nl = 0;
  cs_status st = surround_setup(job, &pl, &kl, &nl);
  if (st) return st;
  *ws_bytes = sv_layout(nl, pl.n_x, n_rows).total;
  return CS_OK;
}

extern "C" cs_status cs_surround(const cs_job* job, const uint32_t* d_bitmap, const uint64_t* d_m, uint64_t n_rows,
                                 cs_surround_row* d_out, void* d_ws, uint64_t ws_bytes, cs_surround_stats* stats,
                                 void* stream) {
  if (!job) return CS_EINVAL;
  if (stats) memset(stats, 0, sizeof *stats);
  if (n_rows >= (1ull << 30)) return CS_ERANGE;
  Plan pl;
  std::vector<uint32_t> kl;
  uint32_t nl = 0;
  cs_status st = surround_setup(job, &pl, &kl, &nl);
  if (st) return st;
  if (n_rows == 0) return CS_OK;
  if (!d_bitmap || !d_m || !d_out || !d_ws) return CS_EINVAL;
  const SvLayout L = sv_layout(nl, pl.n_x, n_rows);
  if (ws_bytes < L.total) return CS_ERANGE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* ws = static_cast<uint8_t*>(d_ws);

  std::vector<int32_t> xs;
  host_columns(pl.job, pl.kq, &xs);
  int32_t c_neg = -1, c_pos = (int32_t)xs.size();
  for (size_t c = 0; c < xs.size(); ++c) {
    if (xs[c] < 0) c_neg = (int32_t)c;
    if (xs[c] > 0 && c_pos == (int32_t)xs.size()) c_pos = (int32_t)c;
  }
  kl.resize(nl, 0u);

  SurroundDev sv;
  sv.bitmap = d_bitmap;
  sv.m = d_m;
  sv.klimbs = reinterpret_cast<const uint32_t*>(ws + L.klimbs);
  sv.x_of_col = reinterpret_cast<const int32_t*>(ws + L.xcol);
  sv.cur = reinterpret_cast<int32_t*>(ws + L.cur);
  sv.nxt = reinterpret_cast<int32_t*>(ws + L.nxt);
  sv.slot_col = reinterpret_cast<int32_t*>(ws + L.slot_col);
  sv.slot_res = ws + L.slot_res;
  sv.act[0] = reinterpret_cast<uint32_t*>(ws + L.act0);
  sv.act[1] = reinterpret_cast<uint32_t*>(ws + L.act1);
  sv.n_act = reinterpret_cast<uint32_t*>(ws + L.n_act);
  sv.tests = reinterpret_cast<unsigned long long*>(ws + L.n_act + 16);
  sv.out = d_out;
  sv.n_rows = n_rows;
  sv.m_lo = pl.job.m_start;
  sv.m_hi = pl.job.m_start + pl.job.m_inc;
  sv.row_words = pl.row_words;
  sv.n_x = pl.n_x;
  sv.c_neg = c_neg;
  sv.c_pos = c_pos;

#define SV_TRY(expr)                                 \
  do {                                               \
    if ((expr) != hipSuccess) return CS_EDEVICE;     \
  } while (0)
  SV_TRY(launch_upload(ws + L.klimbs, kl.data(), nl * 4ull, s));
  if (!xs.empty()) SV_TRY(launch_upload(ws + L.xcol, xs.data(), xs.size() * 4ull, s));
  const uint64_t tasks = 2 * n_rows;
  SV_TRY(launch_fill_u32(sv.n_act, 8, 0u, s));
  hipEvent_t ev[2];
  if (hipEventCreate(&ev[0]) != hipSuccess) return CS_EDEVICE;
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return CS_EDEVICE;
  }
  double test_ms = 0.0, lucas_ms = 0.0;
  uint64_t lucas_passes = 0;
  unsigned long long lucas_run = 0;
  cs_status result = CS_OK;
  uint32_t n_open = (uint32_t)tasks;
  const uint64_t round_target = std::min<uint64_t>(L.slots, sv_resident(nl));
  uint32_t in = 0;
  uint64_t rounds = 0;
  unsigned long long run = 0;
  uint32_t err = 0;
  do {
    hipLaunchKernelGGL(k_sv_init, dim3((uint32_t)((tasks + 255) / 256)), dim3(256), 0, s, sv);
    if (record_launch("k_sv_init") != hipSuccess) { result = CS_EDEVICE; break; }
    for (;;) {
    while (n_open) {
      uint64_t B = std::max<uint64_t>(round_target / n_open, kSurroundB0);
      B = std::min<uint64_t>(std::min<uint64_t>(B, kSurroundBMax), L.slots / n_open);
      const uint32_t b32 = (uint32_t)B;
      const uint32_t g = (n_open + 255) / 256;
      if (launch_fill_u32(sv.n_act + (in ^ 1), 1, 0u, s) != hipSuccess) { result = CS_EDEVICE; break; }
      hipLaunchKernelGGL(k_sv_gather, dim3(g), dim3(256), 0, s, sv, in, n_open, b32);
      if (record_launch("k_sv_gather") != hipSuccess) { result = CS_EDEVICE; break; }
      if (hipEventRecord(ev[0], s) != hipSuccess) { result = CS_EDEVICE; break; }
      if (launch_sv_test(nl, sv, in, (uint64_t)n_open * B, b32, s) != hipSuccess) { result = CS_EDEVICE; break; }
      if (hipEventRecord(ev[1], s) != hipSuccess) { result = CS_EDEVICE; break; }
      hipLaunchKernelGGL(k_sv_resolve, dim3(g), dim3(256), 0, s, sv, in, n_open, b32);
      if (record_launch("k_sv_resolve") != hipSuccess) { result = CS_EDEVICE; break; }
      uint32_t next = 0;
      if (hipMemcpyAsync(&next, sv.n_act + (in ^ 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) { result = CS_EDEVICE; break; }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) test_ms += ms;
      ++rounds;
      n_open = next;
      in ^= 1;
    }
    if (result) break;
    // BPSW: the strong Lucas test of each side's probable prime; the sides whose number fails go
    // back to the rounds from just past it (list `in`), until every found number passes
    if (launch_fill_u32(sv.n_act + in, 1, 0u, s) != hipSuccess) { result = CS_EDEVICE; break; }
    if (hipEventRecord(ev[0], s) != hipSuccess) { result = CS_EDEVICE; break; }
    if (launch_sv_lucas(nl, sv, (uint32_t)kl.size(), in, tasks, s) != hipSuccess) { result = CS_EDEVICE; break; }
    if (hipEventRecord(ev[1], s) != hipSuccess) { result = CS_EDEVICE; break; }
    uint32_t failed = 0;
    if (hipMemcpyAsync(&failed, sv.n_act + in, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { result = CS_EDEVICE; break; }
    float lms = 0.f;
    if (hipEventElapsedTime(&lms, ev[0], ev[1]) == hipSuccess) lucas_ms += lms;
    ++lucas_passes;
    if (failed == 0) break;
    n_open = failed;
    }
    if (result) break;
    if (hipMemcpyAsync(&err, sv.n_act + 2, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&run, sv.tests, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&lucas_run, sv.tests + 1, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      result = CS_EDEVICE;
  } while (0);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
#undef SV_TRY
  if (result) return result;
  if (stats) {
    stats->rounds = rounds;
    stats->tests = run;
    stats->limbs = nl;
    stats->bits = bit_length(kl) + (64 - __builtin_clzll(pl.job.m_start + pl.job.m_inc - 1));
    stats->test_ms = test_ms;
    stats->lucas_tests = lucas_run;
    stats->lucas_passes = lucas_passes;
    stats->lucas_ms = lucas_ms;
  }
  return err ? CS_EDEVICE : CS_OK;
}

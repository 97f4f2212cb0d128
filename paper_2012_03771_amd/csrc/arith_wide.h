// Exact 64-bit residue arithmetic for primes from 2^42 up to 2^63, where the fp64 forms of
// arith.h no longer hold every value exactly (Section 3.3 states the solver for p < 2^64).
//
// Values are unsigned 64-bit integers below p < 2^63; Bezout coefficients are signed 64-bit
// (their magnitude stays below p).  Quotients come from an fp64 estimate of relative error below
// 2^-50: the remainder it leaves, taken with wrapping 64-bit arithmetic, is exact because its true
// magnitude stays below 2^63, and a second fp64 estimate of that small remainder plus one-step
// corrections finish the division.  Products a*b mod p use Montgomery reduction with R = 2^64
// (per-prime constants -p^-1 mod 2^64 and R^2 mod p), which is exact integer arithmetic on the
// 128-bit product.  The descent of Eq. 5, the extended Euclidean pass with the three-gap return
// times, and the driver step are those of arith.h written on these operations.
//
// The functions are __host__ __device__ (the host build is checked against 128-bit integers and
// brute force); the kernels are the only production callers.
#pragma once
#include <stdint.h>
#include <math.h>

#include "arith.h"

namespace cs {

// Full 128-bit product a*b = hi * 2^64 + lo.
CS_HD void mul128(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  *lo = a * b;
  *hi = __umul64hi(a, b);
#else
  const unsigned __int128 t = (unsigned __int128)a * b;
  *lo = (uint64_t)t;
  *hi = (uint64_t)(t >> 64);
#endif
}

// A double estimate of a value in [0, 2^64) clamped so that it converts to uint64_t.
CS_HD uint64_t u64_of(double x) {
  const double top = 18446744073709547520.0;             // 2^64 - 2^12, the largest such double
  x = x < 0.0 ? 0.0 : (x > top ? top : x);
  return (uint64_t)x;
}

// q = floor(a / b), r = a mod b, for a < 2^64 and 1 <= b < 2^63.  For b >= 2^62 the quotient is at
// most 3 and comes from subtractions.  Otherwise the estimate e of a/b has a relative error below
// 2^-50, so |a - floor(e) b| < (1 + a 2^-50 / b) b <= b + 2^14 < 2^63: its wrapping 64-bit value
// is exact as a signed number; a second estimate of that remainder over b and corrections of one
// each way give the exact quotient.
CS_HD void udivmod64(uint64_t a, uint64_t b, uint64_t* q_out, uint64_t* r_out) {
  if (a < b) {
    *q_out = 0;
    *r_out = a;
    return;
  }
  if (b >= (1ull << 62)) {
    uint64_t q = 0;
    while (a >= b) { a -= b; ++q; }
    *q_out = q;
    *r_out = a;
    return;
  }
  const double inv = recip((double)b);
  uint64_t q = u64_of(floor((double)a * inv));
  int64_t r = (int64_t)(a - q * b);
  const double d2 = floor((double)r * inv);              // |r| < 2^63: a small correction
  q += (uint64_t)(int64_t)d2;
  r -= (int64_t)d2 * (int64_t)b;
  if (r < 0) { r += (int64_t)b; --q; }
  if (r < 0) { r += (int64_t)b; --q; }
  if ((uint64_t)r >= b) { r -= (int64_t)b; ++q; }
  if ((uint64_t)r >= b) { r -= (int64_t)b; ++q; }
  *q_out = q;
  *r_out = (uint64_t)r;
}

CS_HD uint64_t umod64(uint64_t a, uint64_t b) {
  uint64_t q, r;
  udivmod64(a, b, &q, &r);
  return r;
}

// (a + b) mod p for a, b < p < 2^63.
CS_HD uint64_t addmod64(uint64_t a, uint64_t b, uint64_t p) {
  const uint64_t s = a + b;
  return s >= p ? s - p : s;
}

// Montgomery constants of an odd modulus 3 <= p < 2^63 with R = 2^64.
struct Mont64 {
  uint64_t p;
  uint64_t np;   // -p^-1 mod 2^64
  uint64_t r2;   // R^2 mod p
};

CS_HD Mont64 mont_setup(uint64_t p) {
  uint64_t x = p;                           // p p == 1 (mod 8): three correct bits
  for (int i = 0; i < 5; ++i) x *= 2 - p * x;   // each Newton step doubles them: 96 >= 64
  Mont64 m;
  m.p = p;
  m.np = 0 - x;
  uint64_t r = umod64(0 - p, p);            // 2^64 mod p
  for (int i = 0; i < 64; ++i) {            // doubled 64 times: 2^128 mod p
    r += r;                                 // r < p < 2^63: no carry
    r = r >= p ? r - p : r;
  }
  m.r2 = r;
  return m;
}

// (hi 2^64 + lo) R^-1 mod p for hi 2^64 + lo < p R.
CS_HD uint64_t redc64(const Mont64& m, uint64_t hi, uint64_t lo) {
  const uint64_t q = lo * m.np;             // lo + q p == 0 (mod 2^64)
  uint64_t mh, ml;
  mul128(q, m.p, &mh, &ml);
  const uint64_t t = hi + mh + (lo != 0 ? 1u : 0u);   // (T + q p) / 2^64 < 2p < 2^64
  return t >= m.p ? t - m.p : t;
}

// a*b mod p for a, b < p: two reductions, the second by R^2 (a b R^-1 R^2 R^-1 = a b).
CS_HD uint64_t mulmod_m(const Mont64& m, uint64_t a, uint64_t b) {
  uint64_t hi, lo;
  mul128(a, b, &hi, &lo);
  const uint64_t x = redc64(m, hi, lo);
  mul128(x, m.r2, &hi, &lo);
  return redc64(m, hi, lo);
}

// k^-1 mod p (gcd(k, p) = 1, 1 <= k < p < 2^63) by the extended Euclidean algorithm.
CS_HD uint64_t modinv64(uint64_t k, uint64_t p) {
  uint64_t a = p, b = k;
  int64_t s0 = 0, s1 = 1;                                 // s_i * k == r_i (mod p)
  for (int it = 0; it < 128 && b != 0; ++it) {
    uint64_t q, r;
    udivmod64(a, b, &q, &r);
    const int64_t s2 = s0 - (int64_t)q * s1;              // |s2| <= p: exact in wrapping arithmetic
    a = b; b = r; s0 = s1; s1 = s2;
  }
  return (uint64_t)(s0 < 0 ? s0 + (int64_t)p : s0);
}

// The offset form of G(p, K, L, R) (Eq. 4-5) of arith.h's g_offset, in 64-bit integers:
// off = v - L for the value v = t K mod p of the least t >= 0 with L <= t K mod p <= L + width.
// Preconditions: gcd(p, K) = 1, 1 <= K < p < 2^63, L + width < p.  Returns ~0 on failure (never
// for valid input).
CS_HD uint64_t g_offset64(uint64_t p, uint64_t K, uint64_t L, uint64_t width, int* levels_out,
                          int max_levels = 256) {
  int par = 0, lv = 0;
  uint64_t off = ~0ull;
  for (; lv < max_levels; ++lv) {
    if (L == 0) { off = 0; break; }                                   // (a)
    if (K >= p - K) {                                                 // (d): 2K >= p
      L = p - L - width;
      K = p - K;
      par ^= 1;
    }
    uint64_t q, rem;
    udivmod64(L, K, &q, &rem);                                        // L mod K
    const uint64_t up = rem == 0 ? 0 : K - rem;                       // ceil(L/K) K - L
    if (up <= width) { off = up; break; }                             // (c)
    const uint64_t pm = umod64(p, K);                                 // p mod K, in (0, K)
    p = K;                                                            // (e)
    K = pm == 0 ? 0 : K - pm;
    L = rem;
    if (K == 0) { off = ~0ull; break; }                               // only if gcd(p, K) > 1
  }
  if (levels_out) *levels_out = lv + 1;
  if (off == ~0ull) return ~0ull;
  return par ? width - off : off;
}

// Smallest t >= 1 with (r + t k) mod p <= w, given r > w; writes the residue reached.  0 on an
// internal failure.
CS_HD uint64_t next_hit64(const Mont64& m, uint64_t k, uint64_t kinv, uint64_t r, uint64_t w, uint64_t* r_new,
                          int* levels) {
  const uint64_t p = m.p;
  const uint64_t L = p - r;                 // t k mod p must lie in [p - r, p - r + w]
  const uint64_t off = g_offset64(p, k, L, w, levels);
  if (off == ~0ull) return 0;
  *r_new = off;                             // (r + v) - p with v = L + off
  return mulmod_m(m, L + off, kinv);
}

// The three-gap constants of the rotation by k mod p for the window [0, w] and k^-1 mod p, from
// one extended Euclidean pass (three_gap_euclid of arith.h in 64-bit integers).  Requires
// 1 <= k < p < 2^63, p prime, 1 <= w, p > 2w.  Returns 0 only on an internal failure.
CS_HD void tg_side64(uint64_t a, uint64_t b, int64_t sa, int64_t sb, uint64_t w, uint64_t* t, uint64_t* v) {
  uint64_t j, rj;
  udivmod64(a - w + b - 1, b, &j, &rj);                       // j = ceil((a - w) / b), a > w
  const uint64_t asb = (uint64_t)(sb < 0 ? -sb : sb), asa = (uint64_t)(sa < 0 ? -sa : sa);
  *t = j * asb + asa;
  *v = a - j * b;                                             // residue on this side, in [1, w]
}

CS_HD int three_gap_euclid64(uint64_t p, uint64_t k, uint64_t w, gaps3* g, uint64_t* kinv_out) {
  uint64_t a = p, b = k;            // r_{i-1}, r_i
  int64_t sa = 0, sb = 1;           // s_{i-1}, s_i
  uint64_t r = 0;
  int64_t sn = 0;
  int it = 0;
  if (b > w) {
    for (; it < 256; ++it) {
      uint64_t q;
      udivmod64(a, b, &q, &r);
      sn = sa - (int64_t)q * sb;
      if (r <= w) break;                                      // the first remainder at or below w
      a = b; b = r; sa = sb; sb = sn;
    }
    if (it == 256) return 0;
  }
  uint64_t t1, v1, t2, v2;
  bool pos1;
  if (b <= w) {                                               // k <= w: t = 1 on the positive side
    t1 = 1;
    v1 = b;
    pos1 = true;
    uint64_t q;
    udivmod64(a, b, &q, &r);
    sn = sa - (int64_t)q * sb;
    tg_side64(a, b, sa, sb, w, &t2, &v2);
  } else {
    pos1 = sa > 0;
    tg_side64(a, b, sa, sb, w, &t1, &v1);
    a = b; b = r; sa = sb; sb = sn;
    uint64_t q;
    udivmod64(a, b, &q, &r);
    sn = sa - (int64_t)q * sb;
    tg_side64(a, b, sa, sb, w, &t2, &v2);
  }
  a = b; b = r; sa = sb; sb = sn;
  for (int i = 0; i < 256 && b != 0; ++i) {                  // the rest, for k^-1 only
    uint64_t q;
    udivmod64(a, b, &q, &r);
    sn = sa - (int64_t)q * sb;
    a = b; b = r; sa = sb; sb = sn;
  }
  if (a != 1) return 0;
  g->ta = pos1 ? t1 : t2;
  g->a = pos1 ? v1 : v2;
  g->tb = pos1 ? t2 : t1;
  g->b = pos1 ? v2 : v1;
  *kinv_out = (uint64_t)(sa < 0 ? sa + (int64_t)p : sa);
  return 1;
}

// K mod p as the product of K's prime groups (each below 2^50) modulo p, for odd p < 2^63.
template <class G>
CS_HD uint64_t kmod64(const Mont64& m, G groups, uint32_t n) {
  uint64_t x = 1 % m.p;
  for (uint32_t t = 0; t < n; ++t) {
    uint64_t g = groups[t];
    if (g >= m.p) g = umod64(g, m.p);
    x = mulmod_m(m, x, g);
  }
  return x;
}

}  // namespace cs

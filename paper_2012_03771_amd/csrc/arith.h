// Exact integer arithmetic for the sieve kernels, written for gfx950's full-rate fp64 VALU.
//
// All residues handled here are below 2^42 (the library's documented sieve-limit range), so
// they are exactly representable as doubles.  Quotients come from an fp64 reciprocal within a
// unit in the last place and are corrected by one exact fma step, so every remainder is exact;
// Euclidean steps on remainders below 2^20 run in fp32 the same way.
// Products beyond 2^53 (a*b mod p) take an fp64 quotient estimate and an exact 64-bit
// wrapping difference (the classic floating-point-quotient modular multiplication).
//
// The functions are __host__ __device__ so the host build can unit-test them against brute
// force; the kernels are the only production callers.
#pragma once
#include <stdint.h>
#include <math.h>

#if defined(__HIPCC__)
#define CS_HD __host__ __device__ __forceinline__
#else
#define CS_HD static inline
#endif

namespace cs {

// 1/x for 1 <= x < 2^52.  On the device: the hardware reciprocal (relative error about 2^-24 on
// gfx950) refined by two Newton steps, each squaring the error, so the result is within a unit
// in the last place (five instructions against eleven for the IEEE division with its scaling and
// fix-up, which positive normal arguments do not need).  Callers only rely on a relative error
// far below 2^-46.  The host build, which only serves tests, moves the correctly rounded quotient
// by one unit in either direction so that the quotient corrections that depend on the rounding
// are exercised.
CS_HD double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  const double r = 1.0 / x;
  const uint64_t h = (uint64_t)x * 0x9E3779B97F4A7C15ull;   // direction by a hash of the argument
  return nextafter(r, (h >> 63) ? 0.0 : 2.0 * r);
#endif
}

// 1/x for 1 <= x < 2^52 with one Newton step: a relative error below 2^-47 (the seed's error
// squared, about 2^-48.8, plus the rounding of the step), three instructions.  For integers
// y, x < 2^42 the product y * recip1(x) is then within (y / x) 2^-47 < 1/x of y/x, whose
// fractional part is 0 or at least 1/x: its floor is exact unless x divides y, when it may be
// one low.  The host build, which only serves tests, moves the correctly rounded quotient by
// 2^-48 of its value in either direction, the size of the device's error.
CS_HD double recip1(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  const double r = 1.0 / x;
  const uint64_t h = (uint64_t)x * 0x9E3779B97F4A7C15ull;   // direction by a hash of the argument
  return (h >> 63) ? r * (1.0 - 0x1p-48) : r * (1.0 + 0x1p-48);
#endif
}

// 1/x in fp32 to within one unit in the last place (the device's hardware reciprocal).  The host
// build, which only serves tests, perturbs the correctly rounded quotient by one unit in either
// direction so that callers are checked against the worst error they allow.
CS_HD float rcp_f32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  const float r = 1.0f / x;
  const uint32_t h = (uint32_t)x * 2654435761u;   // direction by a hash of the (integer) argument
  return nextafterf(r, (h >> 31) ? 0.0f : 2.0f * r);
#endif
}

// The rest of an extended Euclidean pass once the remainders (a, b) are below 2^20, for the
// Bezout coefficients alone: (a, b, sa, sb) with sa*k == a and sb*k == b (mod p) become
// (gcd, 0, s, .) with s*k == gcd (mod p).  Integers below 2^20 are exact in fp32.  The product of
// a and a reciprocal of b within 1.5 units in the last place is within a relative 2^-22 of a/b,
// an absolute error below a * 2^-22 / b < 1/b.  The fractional part of a/b is 0 or at least 1/b,
// so the floor is exact unless b divides a, when it may be one low (remainder b): one exact fma
// and one upward correction give the quotient.  The coefficients stay below p in magnitude and
// are updated in fp64.
CS_HD void euclid_tail_f32(double* a, double* b, double* sa, double* sb) {
  float af = (float)*a, bf = (float)*b;
  double s0 = *sa, s1 = *sb;
  for (int it = 0; it < 64 && bf != 0.0f; ++it) {   // at most 30 steps below 2^20 (Fibonacci)
    float q = floorf(af * rcp_f32(bf));
    float r = fmaf(-q, bf, af);
    if (r >= bf) { r -= bf; q += 1.0f; }
    const double s2 = fma(-(double)q, s1, s0);
    af = bf; bf = r; s0 = s1; s1 = s2;
  }
  *a = (double)af;
  *b = 0.0;
  *sa = s0;
  *sb = s1;
}

// x mod m for 0 <= x < 2^52, 1 <= m < 2^52, with inv = 1/m to a relative error below 2^-46
// and x/m < 2^45: |x/m - x*inv| < 1 so the floor is off by at most one; one exact fma and one
// correction each way make the remainder exact.
CS_HD double fmod_inv(double x, double m, double inv) {
  double q = floor(x * inv);
  double r = fma(-q, m, x);
  r = (r < 0.0) ? r + m : r;
  r = (r >= m) ? r - m : r;
  return r;
}

// a*b mod p for p < 2^52 and a*b/p < 2^50 (a, b need not be reduced).
// pinv = 1/p correctly rounded.  The fp64 quotient is within one of floor(a*b/p); the
// 64-bit wrapping difference a*b - q*p then equals the true (small) remainder.
CS_HD uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p, double pinv) {
  double qd = floor((double)a * (double)b * pinv);
  uint64_t q = (uint64_t)qd;
  int64_t r = (int64_t)(a * b - q * p);
  r = (r < 0) ? r + (int64_t)p : r;
  r = (r >= (int64_t)p) ? r - (int64_t)p : r;
  return (uint64_t)r;
}

// r*g modulo p up to a small multiple of p, in fp64 alone, for |r| < 2.5p, 0 <= g < 2^50,
// p < 2^42 and pinv = 1/p correctly rounded: h + l = r*g exactly (h the rounded product,
// l = fma(r, g, -h) its error, |l| <= |h| 2^-53 < 0.32p); h*pinv is within 0.63 of h/p, so its
// floor q is within one of floor(h/p), h - q*p lies in [-p, 2p) and the fma forms it exactly.
// The result h - q*p + l is an exact integer congruent to r*g with |x| < 2.32p, a valid r again:
// a chain of products needs one full reduction at its end (reduce_f64).
CS_HD double mulmod_f64_lazy(double r, double g, double p, double pinv) {
  const double h = r * g;
  const double l = fma(r, g, -h);
  const double q = floor(h * pinv);
  return fma(-q, p, h) + l;
}

// x mod p in [0, p) for an integer |x| < 2.5p (p < 2^42, pinv = 1/p correctly rounded): the floor
// of x*pinv is within one of floor(x/p), and one correction each way finishes.
CS_HD double reduce_f64(double x, double p, double pinv) {
  const double q = floor(x * pinv);
  double y = fma(-q, p, x);
  y = y < 0.0 ? y + p : y;
  return y >= p ? y - p : y;
}

// r*g mod p in [0, p), for 0 <= r < p < 2^42, 0 <= g < 2^50: one lazy product and one
// reduction, eleven fp64 operations against about three times as many for mulmod's integer
// wrap-around.
CS_HD double mulmod_f64(double r, double g, double p, double pinv) {
  return reduce_f64(mulmod_f64_lazy(r, g, p, pinv), p, pinv);
}

// x mod p for any 64-bit x and p < 2^42.
CS_HD uint64_t mod64(uint64_t x, uint64_t p, double pinv) {
  if (x < (1ull << 52)) return (uint64_t)fmod_inv((double)x, (double)p, pinv);
  uint64_t hi = x >> 32, lo = x & 0xffffffffull;
  uint64_t h = (uint64_t)fmod_inv((double)hi, (double)p, pinv);
  uint64_t t32 = (uint64_t)fmod_inv(4294967296.0, (double)p, pinv);
  uint64_t v = mulmod(h, t32, p, pinv) + (uint64_t)fmod_inv((double)lo, (double)p, pinv);
  return v >= p ? v - p : v;
}

// k^-1 mod p (gcd(k, p) = 1, 1 <= k < p < 2^42) by the extended Euclidean algorithm in
// exact fp64: every remainder and Bezout coefficient stays below p in magnitude.
CS_HD uint64_t modinv(uint64_t k, uint64_t p) {
  double a = (double)p, b = (double)k;
  double s0 = 0.0, s1 = 1.0;          // s_i * k == r_i (mod p)
  for (int it = 0; it < 128 && b != 0.0 && a >= 1048576.0; ++it) {
    double inv = recip1(b);
    double q = floor(a * inv);                 // a < 2^42: exact or one low (as in g_offset)
    double r = fma(-q, b, a);
    if (r >= b) { r -= b; q += 1.0; }
    double s2 = fma(-q, s1, s0);
    a = b; b = r; s0 = s1; s1 = s2;
  }
  euclid_tail_f32(&a, &b, &s0, &s1);  // the remaining steps in fp32, with the lanes reconverged
  // a == gcd == 1 and s0 * k == 1 (mod p)
  double pd = (double)p;
  if (s0 < 0.0) s0 += pd;
  return (uint64_t)s0;
}

// Offset part of the modular-equation solver G(p, K, L, R) of Eq. 4-5: the smallest t >= 0
// with L <= t*K mod p <= R = L + width.  Instead of unwinding the recursion this returns
// off = v - L, where v = t*K mod p is the value the minimal t reaches; the caller recovers
// t = v * K^-1 mod p.  The cases of Eq. 5, one level per pass:
//   (a) L = 0                        -> v = 0.
//   (d) 2K >= p: (p, K, L, R) -> (p, p-K, p-R, p-L); the offset is mirrored: off -> width-off.
//   (c) a multiple of K lies in [L, R] -> v = ceil(L/K)*K, off = K - (L mod K) or 0.
//   (e) (p, K, L, R) -> (K, (-p) mod K, L mod K, R mod K); the offset is unchanged because the
//       solution value satisfies v = floor(L/K)*K + v' with [L, R] free of multiples of K.
// (d) is applied before (c) within a level, by selects, so that a wavefront's lanes follow one
// instruction stream whichever case they are in.  Each case maps the problem to one with the
// same least t (the mirror needs 0 outside [L, R], which (a) guarantees), so the order does
// not change the result.  Case (b) (K >= p) is never met: callers pass K < p and (e) keeps the
// new K below the new p.
// Preconditions: gcd(p, K) = 1, 1 <= K < p < 2^42, 0 <= L, L + width < p.
// Returns -1 (never for valid input) if the descent exceeds `max_levels`.
CS_HD double g_offset(double p, double K, double L, double width, int* levels_out,
                      int max_levels = 160) {
  int par = 0, lv = 0;
  double off = -1.0;
  for (; lv < max_levels; ++lv) {
    // (a) needs no test of its own: with L = 0 the mirror is skipped (it needs 0 outside
    // [L, R]) and (c) finds the multiple 0 of K, offset 0
    const bool mir = K + K >= p && L != 0.0;                   // (d)
    L = mir ? p - L - width : L;
    K = mir ? p - K : K;
    par ^= mir ? 1 : 0;
    // L, p < 2^42 and inv = recip1(K): floor(L*inv) is exact unless K divides L, when it may be
    // one low, so rem lies in [0, K], K standing for 0 (both give up = 0).  gcd(p, K) = 1 at
    // every level ((d) and (e) keep it) and K > 1 here (K = 1 always ends in (c)), so K never
    // divides p: p mod K is exact and in [1, K - 1], and the new K is in [1, K - 1].
    const double inv = recip1(K);
    const double rem = fma(-floor(L * inv), K, L);             // L mod K, or K for 0
    const double up = rem == 0.0 ? 0.0 : K - rem;              // ceil(L/K)*K - L
    if (up <= width) { off = up; break; }                      // (c)
    const double pm = fma(-floor(p * inv), K, p);              // p mod K
    p = K;                                                      // (e)
    K = K - pm;
    L = rem;
  }
  if (levels_out) *levels_out = lv + 1;
  if (off < 0.0) return -1.0;
  return par ? width - off : off;
}

// The moduli of Eq. 5's descent, and whether the mirror (d) applies at each level, depend on
// (p, K) alone, not on L: a prime's walk solves Eq. 3 many times with one (p, K) and different L.
// GCache holds the first kGCache levels of that descent, computed once: the level's K after the
// mirror, its reciprocal and the mirror flags; a solve then spends at each cached level only the
// remainder of L and the test of (c).  The descent of every L ends at the first level whose K
// (after the mirror) is at most width + 1, since a multiple of such a K lies in every window of
// width + 1 integers; the cache stops there.
constexpr int kGCache = 8;
struct GCache {
  double p0;                 // p
  double km[kGCache];        // K of level i after the mirror (the modulus of level i + 1)
  double inv[kGCache];       // recip1(km[i])
  double p_next, K_next;     // (p, K) of level kGCache, when the cache is full
  uint32_t mir;              // bit i: 2K >= p at level i
  int depth;                 // cached levels
};

CS_HD void g_cache_build(double p, double K, double width, GCache* c) {
  c->p0 = p;
  c->mir = 0;
  int depth = 0;
  bool done = false;
  // every level index is a constant after unrolling, so the cache can live in registers
#pragma unroll
  for (int i = 0; i < kGCache; ++i) {
    const bool mir = K + K >= p;
    const double km = mir ? p - K : K;
    const double inv = recip1(km);
    c->km[i] = km;
    c->inv[i] = inv;
    if (!done) {
      if (mir) c->mir |= 1u << i;
      depth = i + 1;
      if (km <= width + 1.0) {
        done = true;                                            // every L ends at this level
      } else {
        const double pm = fma(-floor(p * inv), km, p);          // p mod km, in [1, km - 1]
        p = km;
        K = km - pm;
      }
    }
  }
  c->depth = depth;
  c->p_next = p;
  c->K_next = K;
}

// g_offset(p, K, L, width) from the cached levels (the same cases, in the same order), then the
// descent itself below them.
CS_HD double g_offset_cached(const GCache& c, double L, double width, int* levels_out) {
  int par = 0;
  double p = c.p0;
#pragma unroll
  for (int i = 0; i < kGCache; ++i) {
    if (i < c.depth) {
      const double km = c.km[i];
      const bool mir = ((c.mir >> i) & 1u) != 0 && L != 0.0;   // (d); L = 0 ends in (c) with 0
      L = mir ? p - L - width : L;
      par ^= mir ? 1 : 0;
      const double rem = fma(-floor(L * c.inv[i]), km, L);      // L mod km, or km for 0
      const double up = rem == 0.0 ? 0.0 : km - rem;
      if (up <= width) {                                        // (c)
        if (levels_out) *levels_out = i + 1;
        return par ? width - up : up;
      }
      L = rem;                                                  // (e)
      p = km;
    }
  }
  if (c.depth < kGCache) return -1.0;                           // (never: the cache ended at km <= width + 1)
  int lv = 0;
  const double off = g_offset(c.p_next, c.K_next, L, width, &lv);
  if (levels_out) *levels_out = kGCache + lv;
  if (off < 0.0) return -1.0;
  return par ? width - off : off;
}

// next_hit_d through the cached descent of (p, k).
CS_HD double next_hit_cached(const GCache& c, double kinv, double pinv, double r, double w, double* r_new,
                             int* levels) {
  const double p = c.p0;
  const double L = p - r;
  const double off = g_offset_cached(c, L, w, levels);
  if (off < 0.0) return 0.0;
  *r_new = off;
  return mulmod_f64(L + off, kinv, p, pinv);
}

// Smallest t >= 1 such that (r + t*k) mod p <= w, given r > w (Eq. 3 in shifted form:
// r is the residue of m*K + SL).  Returns t and writes the residue reached (<= w).
// Returns 0 on an internal failure (never for valid input).
CS_HD uint64_t next_hit(uint64_t p, uint64_t k, uint64_t kinv, double pinv, uint64_t r,
                        uint64_t w, uint64_t* r_new, int* levels) {
  double L = (double)(p - r);              // t*k mod p must lie in [p - r, p - r + w]
  double off = g_offset((double)p, (double)k, L, (double)w, levels);
  if (off < 0.0) return 0;
  uint64_t v = (p - r) + (uint64_t)off;    // v = t*k mod p
  *r_new = (uint64_t)off;                  // (r + v) - p
  return mulmod(v, kinv, p, pinv);
}

// next_hit with every value held as a double (all are integers below 2^42): returns t (0.0 on an
// internal failure) and writes the residue reached.  The multiplier is v * k^-1 mod p by
// mulmod_f64, which a reciprocal of p within an ulp serves here: the product v k^-1 < 2^84 over p
// is below 2^42, so h * pinv is within 2^-9 of h / p.
CS_HD double next_hit_d(double p, double k, double kinv, double pinv, double r, double w, double* r_new,
                        int* levels) {
  const double L = p - r;                   // t*k mod p must lie in [p - r, p - r + w]
  const double off = g_offset(p, k, L, w, levels);
  if (off < 0.0) return 0.0;
  *r_new = off;                             // (r + v) - p
  return mulmod_f64(L + off, kinv, p, pinv);
}

// Return-time constants of the rotation by k mod p to the window [0, w] (three-gap theorem):
// ta = least t >= 1 with t*k mod p in [1, w], a = that value;
// tb = least t >= 1 with t*k mod p in [p - w, p - 1], b = p - that value.
// From a hit with residue r (r <= w) the next hit comes after
//   ta      if r + a <= w   (tried first when ta < tb),
//   tb      if r >= b       (tried first when tb < ta),
//   ta + tb otherwise, with residue r + a - b.
// Requires p > 2w so that the two displacement windows do not overlap.
struct gaps3 {
  uint64_t ta, tb, a, b;
};

CS_HD int three_gap_setup(uint64_t p, uint64_t k, uint64_t kinv, double pinv, uint64_t w,
                          gaps3* g, int* levels) {
  int l1 = 0, l2 = 0;
  double oa = g_offset((double)p, (double)k, 1.0, (double)(w - 1), &l1);
  double ob = g_offset((double)p, (double)k, (double)(p - w), (double)(w - 1), &l2);
  if (levels) *levels = l1 + l2;
  if (oa < 0.0 || ob < 0.0) return 0;
  uint64_t va = 1 + (uint64_t)oa, vb = (p - w) + (uint64_t)ob;
  g->a = va;
  g->b = p - vb;
  g->ta = mulmod(va, kinv, p, pinv);
  g->tb = mulmod(vb, kinv, p, pinv);
  return 1;
}

// k^-1 mod p and the three-gap constants of the window [0, w] in one extended Euclidean pass
// over (p, k).  The remainders r_i = s_i * k (mod p) alternate sides: s_i > 0 gives
// t = s_i with t*k mod p = r_i, s_i < 0 gives t = -s_i with t*k mod p = p - r_i.  Along each
// side the one-sided best approximations are the semiconvergents r_{i-1} - j r_i with
// t = |s_{i-1}| + j |s_i|, 1 <= j <= q_i, so the least t whose residue on a side falls to w or
// below is the first such semiconvergent: j = ceil((r_{i-1} - w) / r_i) at the first step whose
// remainder on that side drops to w or below.  The remainders decrease, so the first remainder
// r_{i+1} <= w settles the side of r_{i-1} and the next one, r_{i+2} <= r_{i+1}, the other side:
// the loop runs plain Euclidean steps up to that point and both constants are taken after it
// (when k <= w, t = 1 is the positive side's and the step from (p, k) gives the other).
// Requires 1 <= k < p < 2^42 prime, 1 <= w, p > 2w.  Returns 0 only on an internal failure.
CS_HD void tg_side(double a, double b, double inv, double sa, double sb, double wd, double* t, double* v) {
  const double num = a - wd + b - 1.0;          // j = ceil((a - w) / b), a > w
  double j = floor(num * inv);                  // num < 2^43: exact or one low
  const double rj = fma(-j, b, num);
  j = rj >= b ? j + 1.0 : j;
  *t = fma(j, fabs(sb), fabs(sa));
  *v = fma(-j, b, a);                           // residue on this side, in [1, w]
}

CS_HD int three_gap_euclid(uint64_t p, uint64_t k, uint64_t w, gaps3* g, uint64_t* kinv_out, int* steps_out) {
  const double wd = (double)w;
  double a = (double)p, b = (double)k;        // r_{i-1}, r_i
  double sa = 0.0, sb = 1.0;                  // s_{i-1}, s_i
  double inv = 0.0, r = 0.0, sn = 0.0;
  int it = 0;
  if (b > wd) {
    for (; it < 160; ++it) {
      // b > w >= 1 and gcd(a, b) = 1, so b does not divide a and the floor is exact (recip1)
      inv = recip1(b);
      const double q = floor(a * inv);
      r = fma(-q, b, a);
      sn = fma(-q, sb, sa);                   // s_{i+1}, same side as s_{i-1}
      if (r <= wd) break;                     // the first remainder at or below w
      a = b; b = r; sa = sb; sb = sn;
    }
    if (it == 160) return 0;
  }
  double t1, v1, t2, v2;
  bool pos1;
  if (b <= wd) {                              // k <= w: t = 1 on the positive side
    t1 = 1.0;
    v1 = b;
    pos1 = true;
    inv = recip1(b);                          // (b may be 1 here: the correction stays)
    double q = floor(a * inv);
    r = fma(-q, b, a);
    if (r >= b) { r -= b; q += 1.0; }
    sn = fma(-q, sb, sa);
    tg_side(a, b, inv, sa, sb, wd, &t2, &v2); // negative side from the step (p, k)
  } else {
    pos1 = sa > 0.0;                          // side of r_{i-1} and r_{i+1}
    tg_side(a, b, inv, sa, sb, wd, &t1, &v1);
    // one more exact step: (r_i, r_{i+1}) gives the other side
    a = b; b = r; sa = sb; sb = sn;
    inv = recip1(b);
    double q = floor(a * inv);
    r = fma(-q, b, a);
    if (r >= b) { r -= b; q += 1.0; }
    sn = fma(-q, sb, sa);
    tg_side(a, b, inv, sa, sb, wd, &t2, &v2);
  }
  a = b; b = r; sa = sb; sb = sn;             // a <= w < 2^20
  euclid_tail_f32(&a, &b, &sa, &sb);          // the rest, for k^-1 only, in fp32
  if (steps_out) *steps_out = it;
  // a = gcd = 1 and sa * k == 1 (mod p)
  if (a != 1.0) return 0;
  g->ta = (uint64_t)(pos1 ? t1 : t2);
  g->a = (uint64_t)(pos1 ? v1 : v2);
  g->tb = (uint64_t)(pos1 ? t2 : t1);
  g->b = (uint64_t)(pos1 ? v2 : v1);
  const double pd = (double)p;
  *kinv_out = (uint64_t)(sa < 0.0 ? sa + pd : sa);
  return 1;
}

}  // namespace cs

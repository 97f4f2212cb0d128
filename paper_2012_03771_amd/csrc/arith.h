// Exact integer arithmetic for the sieve kernels, written for gfx950's full-rate fp64 VALU.
//
// All residues handled here are below 2^40 (the library's documented sieve-limit range), so
// they are exactly representable as doubles.  Quotients come from a correctly rounded fp64
// reciprocal and are corrected by one exact fma step, so every remainder is exact.
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

// 1/x, correctly rounded (the IEEE fp64 division; measured faster on gfx950 than a hardware
// reciprocal seed refined by Newton steps inside the dependent chains of the solver).
CS_HD double recip(double x) { return 1.0 / x; }

// x mod m for 0 <= x < 2^52, 1 <= m < 2^52, with inv = 1/m to a relative error below 2^-46
// and x/m < 2^40: |x/m - x*inv| < 1 so the floor is off by at most one; one exact fma and one
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

// x mod p for any 64-bit x and p < 2^40.
CS_HD uint64_t mod64(uint64_t x, uint64_t p, double pinv) {
  if (x < (1ull << 52)) return (uint64_t)fmod_inv((double)x, (double)p, pinv);
  uint64_t hi = x >> 32, lo = x & 0xffffffffull;
  uint64_t h = (uint64_t)fmod_inv((double)hi, (double)p, pinv);
  uint64_t t32 = (uint64_t)fmod_inv(4294967296.0, (double)p, pinv);
  uint64_t v = mulmod(h, t32, p, pinv) + (uint64_t)fmod_inv((double)lo, (double)p, pinv);
  return v >= p ? v - p : v;
}

// k^-1 mod p (gcd(k, p) = 1, 1 <= k < p < 2^40) by the extended Euclidean algorithm in
// exact fp64: every remainder and Bezout coefficient stays below p in magnitude.
CS_HD uint64_t modinv(uint64_t k, uint64_t p) {
  double a = (double)p, b = (double)k;
  double s0 = 0.0, s1 = 1.0;          // s_i * k == r_i (mod p)
  for (int it = 0; it < 128 && b != 0.0; ++it) {
    double inv = recip(b);
    double q = floor(a * inv);
    double r = fma(-q, b, a);
    if (r < 0.0) { r += b; q -= 1.0; }
    if (r >= b) { r -= b; q += 1.0; }
    double s2 = fma(-q, s1, s0);
    a = b; b = r; s0 = s1; s1 = s2;
  }
  // a == gcd == 1 and s0 * k == 1 (mod p)
  double pd = (double)p;
  if (s0 < 0.0) s0 += pd;
  return (uint64_t)s0;
}

// Offset part of the modular-equation solver G(p, K, L, R) of Eq. 4-5: the smallest t >= 0
// with L <= t*K mod p <= R = L + width.  Instead of unwinding the recursion this returns
// off = v - L, where v = t*K mod p is the value the minimal t reaches; the caller recovers
// t = v * K^-1 mod p.  Case by case (first match wins, as in Eq. 5):
//   (a) L = 0                        -> v = 0.
//   (c) a multiple of K lies in [L, R] -> v = ceil(L/K)*K, off = K - (L mod K) or 0.
//   (d) 2K >= p: (p, K, L, R) -> (p, p-K, p-R, p-L); the offset is mirrored: off -> width-off.
//   (e) (p, K, L, R) -> (K, (-p) mod K, L mod K, R mod K); the offset is unchanged because the
//       solution value satisfies v = floor(L/K)*K + v' with [L, R] free of multiples of K.
// Case (b) (K >= p) is never met: callers pass K < p and (e) keeps the new K below the new p.
// Preconditions: gcd(p, K) = 1, 1 <= K < p < 2^40, 0 <= L, L + width < p.
// Returns -1 (never for valid input) if the descent exceeds `max_levels`.
CS_HD double g_offset(double p, double K, double L, double width, int* levels_out,
                      int max_levels = 160) {
  int par = 0, lv = 0;
  double off = -1.0;
  for (; lv < max_levels; ++lv) {
    if (L == 0.0) { off = 0.0; break; }                       // (a)
    double inv = recip(K);
    double rem = fmod_inv(L, K, inv);                          // L mod K
    if (rem == 0.0) { off = 0.0; break; }                      // (c): K | L
    double up = K - rem;                                       // ceil(L/K)*K - L
    if (up <= width) { off = up; break; }                      // (c)
    if (K + K >= p) {                                          // (d)
      L = p - L - width;
      K = p - K;
      par ^= 1;
      continue;
    }
    double pm = fmod_inv(p, K, inv);                           // p mod K (nonzero: gcd = 1)
    p = K;                                                      // (e)
    K = (pm == 0.0) ? 0.0 : K - pm;
    L = rem;
    if (K == 0.0) { off = -1.0; break; }                       // only if gcd(p, K) > 1
  }
  if (levels_out) *levels_out = lv + 1;
  if (off < 0.0) return -1.0;
  return par ? width - off : off;
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
// remainder on that side drops to w or below.  Requires 1 <= k < p < 2^40 prime, 1 <= w,
// p > 2w.  Returns 0 only on an internal failure.
CS_HD int three_gap_euclid(uint64_t p, uint64_t k, uint64_t w, gaps3* g, uint64_t* kinv_out, int* steps_out) {
  const double wd = (double)w;
  double a = (double)p, b = (double)k;        // r_{i-1}, r_i
  double sa = 0.0, sb = 1.0;                  // s_{i-1}, s_i
  bool fa = false, fb = false;                // positive side (t*k mod p small), negative side
  if (b <= wd) {                              // t = 1
    g->ta = 1;
    g->a = k;
    fa = true;
  }
  int it = 0;
  for (; it < 160 && b != 0.0; ++it) {
    const double inv = recip(b);
    double q = floor(a * inv);
    double r = fma(-q, b, a);
    if (r < 0.0) { r += b; q -= 1.0; }
    if (r >= b) { r -= b; q += 1.0; }
    const double sn = fma(-q, sb, sa);        // s_{i+1}, same side as s_{i-1}
    const bool pos = sa > 0.0;                // side of r_{i-1} and r_{i+1} (s_{-1} = 0: negative)
    if (r <= wd && (pos ? !fa : !fb)) {
      double j = floor((a - wd + b - 1.0) * inv);   // ceil((a - w) / b), a > w on this side
      double rem = fma(-j, b, a - wd + b - 1.0);
      if (rem < 0.0) j -= 1.0;
      if (rem >= b) j += 1.0;
      const double t = fabs(sa) + j * fabs(sb);
      const double v = a - j * b;                   // residue on this side, in [1, w]
      if (pos) { g->ta = (uint64_t)t; g->a = (uint64_t)v; fa = true; }
      else { g->tb = (uint64_t)t; g->b = (uint64_t)v; fb = true; }
    }
    a = b; b = r; sa = sb; sb = sn;
  }
  if (steps_out) *steps_out = it;
  // a = gcd = 1 and sa * k == 1 (mod p)
  if (a != 1.0 || !fa || !fb) return 0;
  const double pd = (double)p;
  *kinv_out = (uint64_t)(sa < 0.0 ? sa + pd : sa);
  return 1;
}

}  // namespace cs

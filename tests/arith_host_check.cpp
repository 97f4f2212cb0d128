// Host-side check of the kernels' arithmetic header against brute force.
// Built and run by tests/test_arith_host.py with g++ (the header's functions are plain inline
// C++ outside hipcc).  Exit status 0 means every case agreed.
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_2012_03771_amd/csrc/arith.h"
#include "../paper_2012_03771_amd/csrc/arith_wide.h"

typedef unsigned __int128 u128;

static bool is_prime(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t q = 2; q * q <= n; ++q)
    if (n % q == 0) return false;
  return true;
}

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  for (; e; e >>= 1, b = (uint64_t)((u128)b * b % m))
    if (e & 1) r = (uint64_t)((u128)r * b % m);
  return r;
}

// deterministic Miller-Rabin for 64-bit n (the first twelve prime bases)
static bool is_prime_mr(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t q : bases)
    if (n % q == 0) return n == q;
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s && comp; ++r) {
      x = (uint64_t)((u128)x * x % n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

static uint64_t brute_G(uint64_t p, uint64_t K, uint64_t L, uint64_t R) {
  for (uint64_t m = 0; m < p; ++m) {
    uint64_t v = (uint64_t)((u128)m * K % p);
    if (L <= v && v <= R) return m;
  }
  return ~0ull;
}

static int fail(const char* what, uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
  std::printf("FAIL %s %llu %llu %llu %llu\n", what, (unsigned long long)a, (unsigned long long)b,
              (unsigned long long)c, (unsigned long long)d);
  return 1;
}

int main(int argc, char** argv) {
  unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1;
  std::mt19937_64 rng(seed);
  int bad = 0;

  // mulmod / mod64 / modinv against 128-bit integer arithmetic, p up to 2^42
  for (int i = 0; i < 200000 && !bad; ++i) {
    uint64_t p = (rng() >> (22 + rng() % 40)) | 3;
    if (p >= (1ull << 42)) p &= (1ull << 42) - 1;
    if (p < 3) p = 3;
    double pinv = 1.0 / (double)p;
    uint64_t a = rng() % p, b = rng() % p;
    if (cs::mulmod(a, b, p, pinv) != (uint64_t)((u128)a * b % p)) bad = fail("mulmod", a, b, p, 0);
    uint64_t x = rng();
    if (cs::mod64(x, p, pinv) != x % p) bad = fail("mod64", x, p, 0, 0);
    uint64_t o = rng() & 0xffffffffull;
    if (cs::mulmod(o, a, p, pinv) != (uint64_t)((u128)o * a % p)) bad = fail("mulmod_o", o, a, p, 0);
  }
  // fp64-only modular product for the K mod p chain: r < p < 2^42, g < 2^50
  for (int i = 0; i < 400000 && !bad; ++i) {
    uint64_t p = (rng() >> (22 + rng() % 42)) | 1;
    if (p >= (1ull << 42)) p &= (1ull << 42) - 1;
    if (p < 3) p = 3;
    const uint64_t r = (i % 5 == 0) ? p - 1 - rng() % std::min<uint64_t>(p, 3) : rng() % p;
    uint64_t g = (rng() >> (14 + rng() % 50)) | 1;
    if (g >= (1ull << 50)) g &= (1ull << 50) - 1;
    if (i % 7 == 0) g = (1ull << 50) - 1 - rng() % 1000;
    if (i % 97 == 0) g = 0;                         // K mod p = 0 (p divides K)
    const double pinv = 1.0 / (double)p;
    const double got = cs::mulmod_f64((double)r, (double)g, (double)p, pinv);
    if ((uint64_t)got != (uint64_t)((u128)r * g % p) || got < 0.0) { bad = fail("mulmod_f64", r, g, p, (uint64_t)got); break; }
  }
  // chains of lazily reduced products (the K mod p kernel): |x| stays below 2.32p, and one
  // reduction at the end gives the product of the chain mod p
  for (int i = 0; i < 20000 && !bad; ++i) {
    uint64_t p = (rng() >> (22 + rng() % 42)) | 1;
    if (p >= (1ull << 42)) p &= (1ull << 42) - 1;
    if (i % 9 == 0) p = (1ull << 42) - 1 - 2 * (rng() % 1000);
    if (p < 3) p = 3;
    const double pd = (double)p, pinv = 1.0 / pd;
    const int len = 1 + (int)(rng() % 300);
    double x = 1.0;
    uint64_t want = 1 % p;
    for (int t = 0; t < len && !bad; ++t) {
      uint64_t g = (rng() >> (14 + rng() % 50)) | 1;
      if (g >= (1ull << 50)) g &= (1ull << 50) - 1;
      if (rng() % 3 == 0) g = (1ull << 50) - 1 - rng() % 1000;
      x = cs::mulmod_f64_lazy(x, (double)g, pd, pinv);
      want = (uint64_t)((u128)want * g % p);
      if (!(fabs(x) < 2.32 * pd) || x != floor(x)) bad = fail("mulmod_f64_lazy_bound", p, g, (uint64_t)t, 0);
    }
    const double got = cs::reduce_f64(x, pd, pinv);
    if (!bad && (got < 0.0 || (uint64_t)got != want)) bad = fail("mulmod_f64_lazy_chain", p, want, (uint64_t)got, 0);
  }
  for (int i = 0; i < 20000 && !bad; ++i) {
    uint64_t p;
    do { p = (rng() >> (24 + rng() % 30)) | 1; } while (!is_prime(p));
    uint64_t k = 1 + rng() % (p - 1);
    uint64_t inv = cs::modinv(k, p);
    if ((uint64_t)((u128)inv * k % p) != 1) bad = fail("modinv", k, p, inv, 0);
  }

  // G of Eq. 4 (via the offset form) against brute force on small primes
  for (int i = 0; i < 20000 && !bad; ++i) {
    uint64_t p;
    do { p = 3 + rng() % 20000; } while (!is_prime(p));
    uint64_t K = 1 + rng() % (p - 1);
    uint64_t L = rng() % p;
    uint64_t R = L + rng() % (p - L);
    if (rng() % 4 == 0) R = L + rng() % 4 < p ? L + rng() % 4 : L;
    if (R >= p) R = p - 1;
    uint64_t want = brute_G(p, K, L, R);
    int lv = 0;
    double off = cs::g_offset((double)p, (double)K, (double)L, (double)(R - L), &lv);
    if (off < 0) { bad = fail("g_offset_neg", p, K, L, R); break; }
    uint64_t v = L + (uint64_t)off;
    uint64_t got = (uint64_t)((u128)v * cs::modinv(K, p) % p);
    if (L == 0) got = 0;
    if (got != want) bad = fail("G", p, K, L, R);
  }

  // The driver: every m with (m*k + SL) mod p <= w, enumerated by next_hit and by the
  // three-gap rule, against a direct scan.
  for (int i = 0; i < 3000 && !bad; ++i) {
    uint64_t w = 2 * (1 + rng() % 60);
    uint64_t p;
    do { p = 2 * w + 1 + rng() % 50000; } while (!is_prime(p));
    uint64_t k = 1 + rng() % (p - 1);
    uint64_t kinv = cs::modinv(k, p);
    double pinv = 1.0 / (double)p;
    uint64_t m_inc = 1 + rng() % (4 * p);
    uint64_t r0 = rng() % p;
    std::vector<uint64_t> want, got, got3;
    uint64_t r = r0;
    for (uint64_t o = 0; o < m_inc; ++o) {
      if (r <= w) want.push_back(o);
      r += k; if (r >= p) r -= p;
    }
    // G per hit
    uint64_t o = 0; r = r0;
    while (o < m_inc) {
      if (r > w) {
        uint64_t rn; int lv;
        uint64_t t = cs::next_hit(p, k, kinv, pinv, r, w, &rn, &lv);
        if (t == 0) { bad = fail("next_hit0", p, k, r, w); break; }
        o += t; if (o >= m_inc) break;
        r = rn;
      }
      got.push_back(o);
      o += 1; r += k; if (r >= p) r -= p;
    }
    if (!bad && got != want) bad = fail("driver", p, k, w, m_inc);
    // G per hit with every value a double (the one-solve-per-hit walk of the kernels), the
    // reciprocal of p within an ulp as on the device
    {
      std::vector<uint64_t> gotd;
      const double pd = (double)p, kd = (double)k, kinvd = (double)kinv, wd = (double)w;
      const double pr = cs::recip(pd);
      double od = 0.0, rd = (double)r0;
      while (od < (double)m_inc) {
        if (rd > wd) {
          double rn; int lv;
          const double t = cs::next_hit_d(pd, kd, kinvd, pr, rd, wd, &rn, &lv);
          if (t == 0.0) { bad = fail("next_hit_d0", p, k, (uint64_t)rd, w); break; }
          od += t; if (od >= (double)m_inc) break;
          rd = rn;
        }
        gotd.push_back((uint64_t)od);
        od += 1.0; rd += kd; if (rd >= pd) rd -= pd;
      }
      if (!bad && gotd != want) bad = fail("driver_d", p, k, w, m_inc);
    }
    // three-gap
    cs::gaps3 g; int lv3;
    if (!cs::three_gap_setup(p, k, kinv, pinv, w, &g, &lv3)) { bad = fail("3gap_setup", p, k, w, 0); break; }
    o = 0; r = r0;
    if (r > w) {
      uint64_t rn; int lv;
      uint64_t t = cs::next_hit(p, k, kinv, pinv, r, w, &rn, &lv);
      o = t; r = rn;
    }
    while (o < m_inc) {
      got3.push_back(o);
      bool a_first = g.ta < g.tb;
      if (a_first ? (r + g.a <= w) : !(r >= g.b) && (r + g.a <= w)) { o += g.ta; r += g.a; }
      else if (r >= g.b) { o += g.tb; r -= g.b; }
      else { o += g.ta + g.tb; r = r + g.a - g.b; }
    }
    if (!bad && got3 != want) bad = fail("three_gap", p, k, w, m_inc);
  }
  // the cached descent of Eq. 5 against the plain one: one cache per (p, K), many L
  for (int i = 0; i < 100000 && !bad; ++i) {
    const uint64_t w = 1 + rng() % (i % 4 == 0 ? 8 : 200000);
    uint64_t p;
    do { p = (rng() >> (22 + rng() % 30)) | 1; } while (p <= 2 * w + 1 || p >= (1ull << 42) || !is_prime_mr(p));
    const uint64_t K = 1 + rng() % (p - 1);
    cs::GCache gc;
    cs::g_cache_build((double)p, (double)K, (double)w, &gc);
    for (int q = 0; q < 8 && !bad; ++q) {
      const uint64_t L = (q == 0) ? 0 : rng() % (p - w);
      int l1 = 0, l2 = 0;
      const double a = cs::g_offset((double)p, (double)K, (double)L, (double)w, &l1);
      const double b = cs::g_offset_cached(gc, (double)L, (double)w, &l2);
      if (a != b || l1 != l2) bad = fail("g_cached", p, K, L, w);
    }
  }
  // and against brute force on small primes
  for (int i = 0; i < 20000 && !bad; ++i) {
    const uint64_t w = rng() % 40;
    uint64_t p;
    do { p = 2 * w + 3 + rng() % 3000; } while (!is_prime(p));
    const uint64_t K = 1 + rng() % (p - 1);
    cs::GCache gc;
    cs::g_cache_build((double)p, (double)K, (double)w, &gc);
    const uint64_t L = rng() % (p - w);
    int lv = 0;
    const double off = cs::g_offset_cached(gc, (double)L, (double)w, &lv);
    const uint64_t t = brute_G(p, K, L, L + w);
    if (off < 0.0 || (uint64_t)((u128)t * K % p) != L + (uint64_t)off) bad = fail("g_cached_brute", p, K, L, w);
  }
  // next_hit_d against next_hit for primes up to 2^42
  for (int i = 0; i < 200000 && !bad; ++i) {
    const uint64_t w = 1 + rng() % 200000;
    uint64_t p;
    do { p = (rng() >> (22 + rng() % 20)) | 1; } while (p <= 2 * w + 1 || p >= (1ull << 42) || !is_prime_mr(p));
    const uint64_t k = 1 + rng() % (p - 1);
    const uint64_t kinv = cs::modinv(k, p);
    const uint64_t r = w + 1 + rng() % (p - w - 1);
    uint64_t rn; int lv;
    const uint64_t t = cs::next_hit(p, k, kinv, 1.0 / (double)p, r, w, &rn, &lv);
    double rnd; int lvd;
    const double td = cs::next_hit_d((double)p, (double)k, (double)kinv, cs::recip((double)p), (double)r, (double)w,
                                     &rnd, &lvd);
    if (t == 0 || (uint64_t)td != t || (uint64_t)rnd != rn) bad = fail("next_hit_d", p, k, r, w);
  }
  // one-pass Euclid: inverse and three-gap constants against brute force and the G-based setup
  for (int i = 0; i < 20000 && !bad; ++i) {
    uint64_t w = 1 + rng() % (i % 3 == 0 ? 4 : 3000);
    uint64_t p;
    do { p = 2 * w + 1 + rng() % (i % 5 == 0 ? 200 : 2000000); } while (!is_prime(p));
    uint64_t k = (i % 7 == 0) ? 1 + rng() % std::min<uint64_t>(3, p - 1) : 1 + rng() % (p - 1);
    if (i % 11 == 0) k = p - 1 - rng() % std::min<uint64_t>(3, p - 2);
    cs::gaps3 g1, g2;
    uint64_t kinv = 0;
    int st;
    if (!cs::three_gap_euclid(p, k, w, &g1, &kinv, &st)) { bad = fail("euclid", p, k, w, 0); break; }
    if ((uint64_t)((u128)kinv * k % p) != 1) { bad = fail("euclid_inv", p, k, kinv, 0); break; }
    double pinv = 1.0 / (double)p;
    int lv;
    if (!cs::three_gap_setup(p, k, cs::modinv(k, p), pinv, w, &g2, &lv)) { bad = fail("setup", p, k, w, 0); break; }
    if (g1.ta != g2.ta || g1.a != g2.a || g1.tb != g2.tb || g1.b != g2.b) { bad = fail("euclid_vs_g", p, k, w, g1.ta); break; }
    if (p < 300000) {   // brute force of the definitions
      uint64_t ta = 0, tb = 0;
      for (uint64_t t = 1; t < p && (!ta || !tb); ++t) {
        uint64_t v = (uint64_t)((u128)t * k % p);
        if (!ta && v >= 1 && v <= w) ta = t;
        if (!tb && v >= p - w) tb = t;
      }
      if (ta != g1.ta || tb != g1.tb) { bad = fail("euclid_brute", p, k, w, ta); break; }
    }
  }
  // the same at the sizes of the sieve (primes up to 2^42, windows up to 2^18 - 2), where the
  // Euclidean pass finishes in fp32: inverse exact, constants equal to the G-based setup
  for (int i = 0; i < 20000 && !bad; ++i) {
    uint64_t w = 1 + rng() % (i % 3 == 0 ? 40000 : (1u << 18) - 2);
    uint64_t p;
    do { p = 2 * w + 1 + (rng() >> (22 + rng() % 28)); } while (p >= (1ull << 42) || !is_prime_mr(p));
    uint64_t k = 1 + rng() % (p - 1);
    if (i % 13 == 0) k = 1 + rng() % 5;
    if (i % 17 == 0) k = p - 1 - rng() % 5;
    cs::gaps3 g1, g2;
    uint64_t kinv = 0;
    if (!cs::three_gap_euclid(p, k, w, &g1, &kinv, nullptr)) { bad = fail("euclid_big", p, k, w, 0); break; }
    if ((uint64_t)((u128)kinv * k % p) != 1) { bad = fail("euclid_big_inv", p, k, kinv, 0); break; }
    const uint64_t inv2 = cs::modinv(k, p);
    if ((uint64_t)((u128)inv2 * k % p) != 1) { bad = fail("modinv_big", p, k, inv2, 0); break; }
    double pinv = 1.0 / (double)p;
    int lv;
    if (!cs::three_gap_setup(p, k, inv2, pinv, w, &g2, &lv)) { bad = fail("setup_big", p, k, w, 0); break; }
    if (g1.ta != g2.ta || g1.a != g2.a || g1.tb != g2.tb || g1.b != g2.b) { bad = fail("euclid_vs_g_big", p, k, w, g1.ta); break; }
  }
  // the fp32 tail alone on every pair below 2^11 and on random pairs below 2^20 (gcd and Bezout)
  for (uint64_t a = 1; a < 2048 && !bad; ++a)
    for (uint64_t b = 0; b <= a && !bad; ++b) {
      double x = (double)a, y = (double)b, s0 = 0.0, s1 = 1.0;
      cs::euclid_tail_f32(&x, &y, &s0, &s1);
      uint64_t g = a, h = b;
      while (h) { uint64_t t = g % h; g = h; h = t; }
      if ((uint64_t)x != g) bad = fail("tail_gcd", a, b, (uint64_t)x, g);
    }
  for (int i = 0; i < 200000 && !bad; ++i) {
    // random pairs below 2^20; the coefficients follow the same recurrence as the Bezout pair
    // (u, v) of the integer Euclidean algorithm: s_final = u*s_a + v*s_b, gcd = u*a + v*b
    const uint64_t a = 1 + rng() % ((1u << 20) - 1), b = rng() % (a + 1);
    const int64_t ca = (int64_t)(rng() % (1u << 20)) - (1 << 19), cb = (int64_t)(rng() % (1u << 20)) - (1 << 19);
    int64_t u0 = 1, v0 = 0, u1 = 0, v1 = 1;
    uint64_t g = a, h = b;
    while (h) {
      const int64_t q = (int64_t)(g / h);
      const uint64_t t = g - (uint64_t)q * h;
      g = h; h = t;
      const int64_t u2 = u0 - q * u1, v2 = v0 - q * v1;
      u0 = u1; v0 = v1; u1 = u2; v1 = v2;
    }
    double x = (double)a, y = (double)b, s0 = (double)ca, s1 = (double)cb;
    cs::euclid_tail_f32(&x, &y, &s0, &s1);
    if ((uint64_t)x != g || y != 0.0) { bad = fail("tail_gcd_rand", a, b, (uint64_t)x, g); break; }
    if ((int64_t)s0 != u0 * ca + v0 * cb) { bad = fail("tail_bezout", a, b, (uint64_t)s0, 0); break; }
  }
  // ---- the 64-bit residue arithmetic (primes up to 2^63) ----
  // division: random dividends and divisors of every magnitude, and divisors near 2^62 and 2^63
  for (int i = 0; i < 400000 && !bad; ++i) {
    const uint64_t a = i % 7 == 0 ? ~0ull - rng() % 1000 : rng() >> (rng() % 64);
    uint64_t b = (rng() >> (1 + rng() % 63)) | 1;
    if (i % 11 == 0) b = (1ull << 62) + (rng() % 1000) - 500;
    if (i % 13 == 0) b = (1ull << 63) - 1 - rng() % 100000;
    if (b >= (1ull << 63)) b = (1ull << 63) - 1;
    uint64_t q, r;
    cs::udivmod64(a, b, &q, &r);
    if (q != a / b || r != a % b) bad = fail("udivmod64", a, b, q, r);
  }
  // Montgomery products, inverses and K mod p against 128-bit integers, odd p up to 2^63
  for (int i = 0; i < 200000 && !bad; ++i) {
    uint64_t p = ((rng() >> (1 + rng() % 60)) | 1) | 3;
    if (i % 9 == 0) p = (1ull << 63) - 1 - 2 * (rng() % 1000);
    const cs::Mont64 m = cs::mont_setup(p);
    const uint64_t a = rng() % p, b = rng() % p;
    if (cs::mulmod_m(m, a, b) != (uint64_t)((u128)a * b % p)) { bad = fail("mulmod_m", a, b, p, 0); break; }
  }
  for (int i = 0; i < 20000 && !bad; ++i) {
    uint64_t p;
    do { p = (rng() >> (1 + rng() % 40)) | 1; } while (p < 5 || !is_prime_mr(p));
    const uint64_t k = 1 + rng() % (p - 1);
    const uint64_t inv = cs::modinv64(k, p);
    if ((uint64_t)((u128)inv * k % p) != 1) { bad = fail("modinv64", p, k, inv, 0); break; }
    const uint64_t gr[4] = {rng() >> 14, rng() >> 14, rng() >> 20, 3};
    uint64_t want = 1 % p;
    for (int t = 0; t < 4; ++t) want = (uint64_t)((u128)want * (gr[t] % p) % p);
    const cs::Mont64 m = cs::mont_setup(p);
    if (cs::kmod64(m, gr, 4) != want) { bad = fail("kmod64", p, gr[0], gr[1], 0); break; }
  }
  // Eq. 5 in 64-bit integers against brute force (small p) and against the fp64 form (p < 2^42)
  for (int i = 0; i < 20000 && !bad; ++i) {
    uint64_t p;
    do { p = 3 + rng() % 4000; } while (!is_prime(p));
    const uint64_t K = 1 + rng() % (p - 1), width = rng() % (p / 2), L = 1 + rng() % (p - width - 1);
    int lv;
    const uint64_t off = cs::g_offset64(p, K, L, width, &lv);
    const uint64_t t = brute_G(p, K, L, L + width);
    const uint64_t v = (uint64_t)((u128)t * K % p);
    if (off == ~0ull || L + off != v) { bad = fail("g_offset64", p, K, L, width); break; }
  }
  for (int i = 0; i < 50000 && !bad; ++i) {
    uint64_t p;
    do { p = (rng() >> (22 + rng() % 20)) | 1; } while (p < (1ull << 20) || !is_prime_mr(p));
    if (p >= (1ull << 42)) continue;
    const uint64_t K = 1 + rng() % (p - 1), width = 1 + rng() % (1u << 17), L = 1 + rng() % (p - width - 1);
    int l1, l2;
    const uint64_t o1 = cs::g_offset64(p, K, L, width, &l1);
    const double o2 = cs::g_offset((double)p, (double)K, (double)L, (double)width, &l2);
    if (o2 < 0.0 || o1 != (uint64_t)o2) { bad = fail("g_offset64_vs_fp64", p, K, L, width); break; }
  }
  // three-gap constants in 64-bit integers: against the fp64 pass below 2^42, and at 2^50..2^63
  // the rule's next hit from a hit against an Eq. 5 solve from the following residue
  for (int i = 0; i < 40000 && !bad; ++i) {
    uint64_t p;
    const int top = i % 2 ? 42 : 63;
    do { p = (rng() >> (64 - top + rng() % 20)) | 1; } while (p < (1ull << 22) || !is_prime_mr(p));
    if (p >= (1ull << 63)) continue;
    const uint64_t w = 1 + rng() % (1u << 18);
    const uint64_t k = 1 + rng() % (p - 1);
    cs::gaps3 g;
    uint64_t kinv = 0;
    if (!cs::three_gap_euclid64(p, k, w, &g, &kinv)) { bad = fail("euclid64", p, k, w, 0); break; }
    if ((uint64_t)((u128)kinv * k % p) != 1) { bad = fail("euclid64_inv", p, k, kinv, 0); break; }
    if ((uint64_t)((u128)g.ta * k % p) != g.a || g.a < 1 || g.a > w) { bad = fail("euclid64_ta", p, k, w, g.ta); break; }
    if (p - (uint64_t)((u128)g.tb * k % p) != g.b || g.b < 1 || g.b > w) { bad = fail("euclid64_tb", p, k, w, g.tb); break; }
    if (p < (1ull << 42)) {
      cs::gaps3 g2;
      uint64_t kinv2 = 0;
      if (!cs::three_gap_euclid(p, k, w, &g2, &kinv2, nullptr) || g2.ta != g.ta || g2.tb != g.tb || g2.a != g.a ||
          g2.b != g.b || kinv2 != kinv) {
        bad = fail("euclid64_vs_fp64", p, k, w, 0);
        break;
      }
    }
    const cs::Mont64 m = cs::mont_setup(p);
    for (int j = 0; j < 4 && !bad; ++j) {
      const uint64_t r = rng() % (w + 1);                     // a hit's residue
      const bool a_first = g.ta < g.tb;
      const bool fa = r + g.a <= w, fb = r >= g.b;
      const uint64_t t_rule = (fa && (a_first || !fb)) ? g.ta : (fb ? g.tb : g.ta + g.tb);
      uint64_t r1 = r + k;                                     // residue after one step
      r1 = r1 >= p ? r1 - p : r1;
      uint64_t t_g = 1, rn = r1;
      int lv;
      if (r1 > w) t_g = 1 + cs::next_hit64(m, k, kinv, r1, w, &rn, &lv);
      if (t_g != t_rule) { bad = fail("three_gap64_vs_G", p, k, r, t_rule); break; }
      if ((uint64_t)(((u128)r + (u128)t_g * k) % p) != rn || rn > w) { bad = fail("next_hit64", p, k, r, t_g); break; }
    }
  }
  if (!bad) std::printf("OK\n");
  return bad;
}

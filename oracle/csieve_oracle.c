/*
 * Plain CPU oracle for the Combined Sieve (test infrastructure only).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library.  It shares no code with the HIP library: its own bignum, its own prime sieve, its
 * own column and row sets.
 *
 * What it computes is the plain definition of the sieve (Section 2.1, traditional sieve, and
 * the interval definition S = 2X + 1 of Section 3.2):
 *
 *   K = P#/d,  rows m in [m_start, m_start + m_inc) with gcd(m, d) = 1,
 *   columns X in [-sl, sl] with gcd(X, K) = 1,
 *   bit[m][X]  = 1  iff some prime p <= limit divides m*K + X,
 *   count[m]   = number of (p, X) pairs, X a column, p <= limit prime, p | m*K + X.
 *
 * For every row and every prime p it takes r = N mod p, N = m*K, and marks the offsets
 * X = -r (mod p) of the interval, exactly as the traditional sieve of Section 2.1 does.
 * Two ways of taking r are offered:
 *   ORC_DIRECT  r = N mod p from the bignum N itself (the literal traditional sieve);
 *   ORC_CACHED  r = ((m mod p) * (K mod p)) mod p, the identity of Eq. 1 (Section 3.1).
 * Both reduce with 128-bit integer '%' and nothing else; no blocking or reordering beyond the
 * loop over primes in blocks of consecutive integers.
 *
 * Output layout: row r (r-th coprime m in the given list), column c (c-th coprime X counted
 * from -sl upwards), word r*row_words + c/32, bit c%32, row_words = ceil(n_x/32).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

typedef unsigned __int128 u128;

enum { ORC_DIRECT = 0, ORC_CACHED = 1 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -3 };

/* ------------------------------------------------------------------------------------- */
/* Bignum: little-endian 64-bit limbs.                                                   */
/* ------------------------------------------------------------------------------------- */
typedef struct {
    uint64_t *w;
    int n;      /* limbs in use */
    int cap;
} big;

static int big_init(big *a, int cap) {
    a->w = (uint64_t *)calloc((size_t)cap, sizeof(uint64_t));
    a->n = 1;
    a->cap = cap;
    if (!a->w) return ORC_ENOMEM;
    a->w[0] = 1;
    return ORC_OK;
}

static void big_free(big *a) { free(a->w); a->w = NULL; }

static void big_mul_u64(big *a, uint64_t m) {
    u128 carry = 0;
    for (int i = 0; i < a->n; ++i) {
        u128 t = (u128)a->w[i] * m + carry;
        a->w[i] = (uint64_t)t;
        carry = t >> 64;
    }
    if (carry) a->w[a->n++] = (uint64_t)carry;
}

/* a /= q in place, returns the remainder */
static uint64_t big_divmod_u64(big *a, uint64_t q) {
    u128 r = 0;
    for (int i = a->n - 1; i >= 0; --i) {
        u128 cur = (r << 64) | a->w[i];
        a->w[i] = (uint64_t)(cur / q);
        r = cur % q;
    }
    while (a->n > 1 && a->w[a->n - 1] == 0) a->n--;
    return (uint64_t)r;
}

/* a mod q by Horner's rule from the most significant limb */
static uint64_t big_mod_u64(const big *a, uint64_t q) {
    u128 r = 0;
    for (int i = a->n - 1; i >= 0; --i) r = ((r << 64) | a->w[i]) % q;
    return (uint64_t)r;
}

static int is_prime_td(uint64_t n) {
    if (n < 2) return 0;
    for (uint64_t q = 2; q * q <= n; ++q)
        if (n % q == 0) return 0;
    return 1;
}

static uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}

/* K = P#/d.  Fails when d does not divide P# or is not squarefree. */
static int make_K(uint32_t P, uint64_t d, big *K) {
    if (P < 2 || d == 0) return ORC_EINVAL;
    int cap = (int)(P / 32) + 4;   /* log2(P#) < 1.45 P bits */
    if (big_init(K, cap) != ORC_OK) return ORC_ENOMEM;
    for (uint32_t q = 2; q <= P; ++q)
        if (is_prime_td(q)) big_mul_u64(K, q);
    /* d must be squarefree and divide P#: remove its prime factors one by one */
    uint64_t rest = d;
    for (uint64_t q = 2; q <= P && rest > 1; ++q) {
        if (rest % q == 0) {
            rest /= q;
            if (rest % q == 0) { big_free(K); return ORC_EINVAL; }
        }
    }
    if (rest != 1) { big_free(K); return ORC_EINVAL; }
    if (big_divmod_u64(K, d) != 0) { big_free(K); return ORC_EINVAL; }
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------- */
/* Primes: base primes by a plain sieve, then a segmented sieve of Eratosthenes.         */
/* ------------------------------------------------------------------------------------- */
#define ORC_SEG (1u << 22)

typedef struct {
    uint32_t *base;     /* primes <= sqrt(hi) */
    size_t nbase;
} base_primes;

static int base_primes_make(uint64_t hi, base_primes *bp) {
    uint64_t r = (uint64_t)sqrtl((long double)hi) + 2;
    while (r * r > hi && r > 0) --r;
    uint64_t n = r + 1;
    uint8_t *comp = (uint8_t *)calloc((size_t)n + 1, 1);
    bp->base = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)n + 1));
    if (!comp || !bp->base) { free(comp); free(bp->base); return ORC_ENOMEM; }
    bp->nbase = 0;
    for (uint64_t i = 2; i <= r; ++i) {
        if (comp[i]) continue;
        bp->base[bp->nbase++] = (uint32_t)i;
        for (uint64_t j = i * i; j <= r; j += i) comp[j] = 1;
    }
    free(comp);
    return ORC_OK;
}

/* Primes in [a, b] (b - a < ORC_SEG) into out; returns how many. */
static size_t sieve_segment(uint64_t a, uint64_t b, const base_primes *bp, uint8_t *comp,
                            uint64_t *out) {
    if (b < a) return 0;
    uint64_t len = b - a + 1;
    memset(comp, 0, (size_t)len);
    for (size_t i = 0; i < bp->nbase; ++i) {
        uint64_t q = bp->base[i];
        if (q * q > b) break;
        uint64_t start = ((a + q - 1) / q) * q;
        if (start < q * q) start = q * q;
        for (uint64_t j = start; j <= b; j += q) comp[j - a] = 1;
    }
    size_t n = 0;
    for (uint64_t i = 0; i < len; ++i) {
        uint64_t v = a + i;
        if (v >= 2 && !comp[i]) out[n++] = v;
    }
    return n;
}

typedef struct {
    uint64_t *primes;
    uint64_t *kmod;     /* K mod p, ORC_CACHED only */
    uint8_t *comp;
    size_t n;
} thread_block;

static int blocks_alloc(thread_block *tb, int nt, int need_k) {
    for (int t = 0; t < nt; ++t) {
        tb[t].primes = (uint64_t *)malloc(sizeof(uint64_t) * ORC_SEG);
        tb[t].comp = (uint8_t *)malloc(ORC_SEG);
        tb[t].kmod = need_k ? (uint64_t *)malloc(sizeof(uint64_t) * ORC_SEG) : NULL;
        tb[t].n = 0;
        if (!tb[t].primes || !tb[t].comp || (need_k && !tb[t].kmod)) return ORC_ENOMEM;
    }
    return ORC_OK;
}

static void blocks_free(thread_block *tb, int nt) {
    for (int t = 0; t < nt; ++t) {
        free(tb[t].primes);
        free(tb[t].comp);
        free(tb[t].kmod);
    }
}

static int pick_threads(int threads) {
    return threads > 0 ? threads : omp_get_max_threads();
}

/* Number of primes in [lo, hi] and the sum of log(1 - 1/p) over them. */
int orc_prime_stats(uint64_t lo, uint64_t hi, uint64_t *count, double *sum_log1m, int threads) {
    if (hi < lo) { *count = 0; *sum_log1m = 0; return ORC_OK; }
    int nt = pick_threads(threads);
    base_primes bp;
    if (base_primes_make(hi, &bp) != ORC_OK) return ORC_ENOMEM;
    thread_block *tb = (thread_block *)calloc((size_t)nt, sizeof(thread_block));
    if (!tb || blocks_alloc(tb, nt, 0) != ORC_OK) {
        if (tb) blocks_free(tb, nt);
        free(tb); free(bp.base);
        return ORC_ENOMEM;
    }
    uint64_t total = 0;
    long double acc = 0.0L;
    for (uint64_t base = lo; base <= hi; base += (uint64_t)nt * ORC_SEG) {
        uint64_t tot_here = 0;
        long double acc_here = 0.0L;
#pragma omp parallel num_threads(nt) reduction(+ : tot_here) reduction(+ : acc_here)
        {
            int t = omp_get_thread_num();
            uint64_t a = base + (uint64_t)t * ORC_SEG;
            if (a >= base && a <= hi) {
                uint64_t b = a + ORC_SEG - 1;
                if (b > hi || b < a) b = hi;
                size_t n = sieve_segment(a, b, &bp, tb[t].comp, tb[t].primes);
                tot_here += n;
                for (size_t i = 0; i < n; ++i) acc_here += log1pl(-1.0L / (long double)tb[t].primes[i]);
            }
        }
        total += tot_here;
        acc += acc_here;
        if (base + (uint64_t)nt * ORC_SEG < base) break;
    }
    *count = total;
    *sum_log1m = (double)acc;
    blocks_free(tb, nt);
    free(tb);
    free(bp.base);
    return ORC_OK;
}

/* Primes in [lo, hi] written to out (at most cap); returns the number of primes in range. */
int64_t orc_primes_range(uint64_t lo, uint64_t hi, uint64_t *out, uint64_t cap) {
    if (hi < lo) return 0;
    base_primes bp;
    if (base_primes_make(hi, &bp) != ORC_OK) return ORC_ENOMEM;
    uint8_t *comp = (uint8_t *)malloc(ORC_SEG);
    uint64_t *buf = (uint64_t *)malloc(sizeof(uint64_t) * ORC_SEG);
    if (!comp || !buf) { free(comp); free(buf); free(bp.base); return ORC_ENOMEM; }
    int64_t total = 0;
    for (uint64_t a = lo; a <= hi; a += ORC_SEG) {
        uint64_t b = a + ORC_SEG - 1;
        if (b > hi || b < a) b = hi;
        size_t n = sieve_segment(a, b, &bp, comp, buf);
        for (size_t i = 0; i < n; ++i) {
            if ((uint64_t)total < cap) out[total] = buf[i];
            ++total;
        }
        if (b == hi) break;
    }
    free(comp); free(buf); free(bp.base);
    return total;
}

/* ------------------------------------------------------------------------------------- */
/* Columns and rows.                                                                      */
/* ------------------------------------------------------------------------------------- */

/* Column set: X in [-sl, sl] with gcd(X, K) = 1, ascending.  col_of[X + sl] = column or -1. */
static int64_t build_columns(const big *K, uint32_t sl, int32_t *col_of, int32_t *x_of_col) {
    int64_t n = 0;
    int K_is_one = (K->n == 1 && K->w[0] == 1);
    for (int64_t X = -(int64_t)sl; X <= (int64_t)sl; ++X) {
        int coprime;
        if (X == 0) {
            coprime = K_is_one;                 /* gcd(0, K) = K */
        } else {
            uint64_t ax = (uint64_t)(X < 0 ? -X : X);
            coprime = gcd_u64(ax, big_mod_u64(K, ax)) == 1;
        }
        if (col_of) col_of[X + sl] = coprime ? (int32_t)n : -1;
        if (coprime) {
            if (x_of_col) x_of_col[n] = (int32_t)X;
            ++n;
        }
    }
    return n;
}

int64_t orc_columns(uint32_t P, uint64_t d, uint32_t sl, int32_t *x_of_col, uint64_t cap) {
    big K;
    int st = make_K(P, d, &K);
    if (st) return st;
    int64_t n = build_columns(&K, sl, NULL, NULL);
    if (x_of_col && (uint64_t)n <= cap) build_columns(&K, sl, NULL, x_of_col);
    big_free(&K);
    return n;
}

/* Rows: m in [m_start, m_start + m_inc) with gcd(m, d) = 1, ascending. */
int64_t orc_rows(uint64_t d, uint64_t m_start, uint64_t m_inc, uint64_t *m_of_row, uint64_t cap) {
    int64_t n = 0;
    for (uint64_t i = 0; i < m_inc; ++i) {
        uint64_t m = m_start + i;
        if (gcd_u64(m, d) == 1) {
            if (m_of_row && (uint64_t)n < cap) m_of_row[n] = m;
            ++n;
        }
    }
    return n;
}

/* ------------------------------------------------------------------------------------- */
/* The sieve: every listed row against every prime in [p_lo, p_hi].                      */
/* ------------------------------------------------------------------------------------- */

/* Marks row `r` for prime p given rr = N mod p. */
static inline void mark_row(uint64_t p, uint64_t rr, uint32_t sl, const int32_t *col_of,
                            uint32_t *bits_row, uint32_t *count, uint64_t *wit_row) {
    /* X = -rr (mod p); j = X + sl = (sl - rr) mod p */
    uint64_t j = ((uint64_t)sl % p + p - rr) % p;
    uint64_t w = 2ull * sl;
    for (; j <= w; j += p) {
        int32_t c = col_of[j];
        if (c < 0) continue;
        bits_row[c >> 5] |= 1u << (c & 31);
        *count += 1;
        if (wit_row && (wit_row[c] == 0 || p < wit_row[c])) wit_row[c] = p;
    }
}

/*
 * rows: explicit list of n_rows multipliers (each must be coprime to d for the result to be a
 * sieve row; the oracle does not filter them).  bits: n_rows * row_words words; counts: n_rows;
 * witness: n_rows * n_x (smallest marking prime per bit, 0 = unmarked) or NULL.
 * All outputs are overwritten.
 */
int orc_sieve_rows(uint32_t P, uint64_t d, uint32_t sl, const uint64_t *rows, uint64_t n_rows,
                   uint64_t p_lo, uint64_t p_hi, int mode, uint32_t *bits, uint32_t *counts,
                   uint64_t *witness, int threads) {
    if (mode != ORC_DIRECT && mode != ORC_CACHED) return ORC_EINVAL;
    big K;
    int st = make_K(P, d, &K);
    if (st) return st;
    uint64_t S = 2ull * sl + 1;
    int32_t *col_of = (int32_t *)malloc(sizeof(int32_t) * S);
    if (!col_of) { big_free(&K); return ORC_ENOMEM; }
    int64_t n_x = build_columns(&K, sl, col_of, NULL);
    uint64_t row_words = ((uint64_t)n_x + 31) / 32;
    memset(bits, 0, sizeof(uint32_t) * row_words * n_rows);
    memset(counts, 0, sizeof(uint32_t) * n_rows);
    if (witness) memset(witness, 0, sizeof(uint64_t) * (uint64_t)n_x * n_rows);
    if (p_lo < 2) p_lo = 2;

    /* N = m*K for every row (ORC_DIRECT) */
    big *N = NULL;
    if (mode == ORC_DIRECT) {
        N = (big *)calloc(n_rows ? n_rows : 1, sizeof(big));
        if (!N) { free(col_of); big_free(&K); return ORC_ENOMEM; }
        for (uint64_t r = 0; r < n_rows; ++r) {
            if (big_init(&N[r], K.n + 2) != ORC_OK) { st = ORC_ENOMEM; break; }
            memcpy(N[r].w, K.w, sizeof(uint64_t) * (size_t)K.n);
            N[r].n = K.n;
            big_mul_u64(&N[r], rows[r]);
        }
    }

    int nt = pick_threads(threads);
    base_primes bp = {0, 0};
    thread_block *tb = NULL;
    if (st == ORC_OK && p_hi >= p_lo && n_rows > 0) {
        st = base_primes_make(p_hi, &bp);
        tb = (thread_block *)calloc((size_t)nt, sizeof(thread_block));
        if (st == ORC_OK && (!tb || blocks_alloc(tb, nt, mode == ORC_CACHED) != ORC_OK)) st = ORC_ENOMEM;
    }
    if (st == ORC_OK && p_hi >= p_lo && n_rows > 0) {
        for (uint64_t base = p_lo; base <= p_hi; base += (uint64_t)nt * ORC_SEG) {
#pragma omp parallel num_threads(nt)
            {
                int t = omp_get_thread_num();
                uint64_t a = base + (uint64_t)t * ORC_SEG;
                tb[t].n = 0;
                if (a >= base && a <= p_hi) {
                    uint64_t b = a + ORC_SEG - 1;
                    if (b > p_hi || b < a) b = p_hi;
                    tb[t].n = sieve_segment(a, b, &bp, tb[t].comp, tb[t].primes);
                    if (mode == ORC_CACHED)
                        for (size_t i = 0; i < tb[t].n; ++i) tb[t].kmod[i] = big_mod_u64(&K, tb[t].primes[i]);
                }
            }
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
            for (uint64_t r = 0; r < n_rows; ++r) {
                uint32_t *brow = bits + r * row_words;
                uint64_t *wrow = witness ? witness + r * (uint64_t)n_x : NULL;
                for (int t = 0; t < nt; ++t) {
                    for (size_t i = 0; i < tb[t].n; ++i) {
                        uint64_t p = tb[t].primes[i];
                        uint64_t rr;
                        if (mode == ORC_DIRECT)
                            rr = big_mod_u64(&N[r], p);
                        else
                            rr = (uint64_t)(((u128)(rows[r] % p) * tb[t].kmod[i]) % p);
                        mark_row(p, rr, sl, col_of, brow, &counts[r], wrow);
                    }
                }
            }
            if (base + (uint64_t)nt * ORC_SEG < base) break;
        }
    }
    if (tb) blocks_free(tb, nt);
    free(tb);
    free(bp.base);
    if (N) {
        for (uint64_t r = 0; r < n_rows; ++r) big_free(&N[r]);
        free(N);
    }
    free(col_of);
    big_free(&K);
    return st;
}

/*
 * Number of primes p in [p_lo, p_hi] that divide at least one of the S = 2*sl + 1 integers
 * N + X, |X| <= sl, N = m*K (every X, coprime to K or not).  Literal: N mod p from the bignum.
 */
int64_t orc_window_hit_primes(uint32_t P, uint64_t d, uint64_t m, uint32_t sl, uint64_t p_lo,
                              uint64_t p_hi, int threads) {
    big N;
    int st = make_K(P, d, &N);
    if (st) return st;
    big_mul_u64(&N, m);   /* capacity has spare limbs */
    if (p_lo < 2) p_lo = 2;
    int nt = pick_threads(threads);
    base_primes bp;
    if (base_primes_make(p_hi, &bp) != ORC_OK) { big_free(&N); return ORC_ENOMEM; }
    thread_block *tb = (thread_block *)calloc((size_t)nt, sizeof(thread_block));
    if (!tb || blocks_alloc(tb, nt, 0) != ORC_OK) {
        if (tb) blocks_free(tb, nt);
        free(tb); free(bp.base); big_free(&N);
        return ORC_ENOMEM;
    }
    int64_t hits = 0;
    uint64_t w = 2ull * sl;
    for (uint64_t base = p_lo; base <= p_hi; base += (uint64_t)nt * ORC_SEG) {
        int64_t here = 0;
#pragma omp parallel num_threads(nt) reduction(+ : here)
        {
            int t = omp_get_thread_num();
            uint64_t a = base + (uint64_t)t * ORC_SEG;
            if (a >= base && a <= p_hi) {
                uint64_t b = a + ORC_SEG - 1;
                if (b > p_hi || b < a) b = p_hi;
                size_t n = sieve_segment(a, b, &bp, tb[t].comp, tb[t].primes);
                for (size_t i = 0; i < n; ++i) {
                    uint64_t p = tb[t].primes[i];
                    uint64_t rr = big_mod_u64(&N, p);
                    uint64_t j = ((uint64_t)sl % p + p - rr) % p;
                    if (j <= w) here += 1;
                }
            }
        }
        hits += here;
        if (base + (uint64_t)nt * ORC_SEG < base) break;
    }
    blocks_free(tb, nt);
    free(tb); free(bp.base); big_free(&N);
    return hits;
}

/* N mod p for N = m*K (used by witness checks on sampled bits). */
int orc_n_mod(uint32_t P, uint64_t d, uint64_t m, const uint64_t *ps, uint64_t n, uint64_t *out) {
    big N;
    int st = make_K(P, d, &N);
    if (st) return st;
    big_mul_u64(&N, m);
    for (uint64_t i = 0; i < n; ++i) out[i] = big_mod_u64(&N, ps[i]);
    big_free(&N);
    return ORC_OK;
}

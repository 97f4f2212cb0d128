/*
 * csieve.h -- C ABI of the MI355X (gfx950) Combined Sieve library.
 *
 * The problem (Section 3 of "Combined Sieve Algorithm for Prime Gaps", S. Troisi,
 * arXiv 2012.03771): for K = P#/d and many multipliers m, sieve the intervals around
 * N = m*K with every prime up to the sieve limit.  Concretely, for a job
 * (P, d, m_start, m_inc, sl, limit):
 *
 *   rows     m in [m_start, m_start + m_inc) with gcd(m, d) = 1 (Section 3: only m coprime
 *            to d are searched; their number is the paper's M_c),
 *   columns  X in [-sl, sl] with gcd(X, K) = 1 (the interval of size S = 2X + 1 of
 *            Section 3.2; offsets sharing a factor with K are composite by construction,
 *            Section 2 "Primorials"),
 *   bit      1 iff some prime p <= limit divides m*K + X,
 *   count    per row, the number of pairs (p, X), p <= limit prime, X a column,
 *            p | m*K + X (every factor the sieve enumerates, Section 3.2).
 *
 * Output layout (all rows and columns ascending):
 *   bitmap   uint32 words; row r, column c at word r*row_words + c/32, bit c%32
 *            (LSB first), row_words = ceil(n_x/32); padding bits are 0.
 *   counts   uint32[n_m].
 *
 * Conventions for every entry point:
 *   - Device buffers (d_*) belong to the caller and must stay valid until the work
 *     enqueued on `stream` has completed.  `stream` is a hipStream_t (NULL = legacy default
 *     stream).  Calls enqueue work and return without waiting unless stated otherwise.
 *   - Arguments are validated before anything is enqueued; on any error nothing is enqueued
 *     and the outputs are untouched.  No entry point prints, throws or aborts.
 *   - Faults of enqueued work surface as CS_EDEVICE from the next call that synchronises
 *     (cs_diag_read, cs_server_*); outputs are then undefined.
 *   - The library allocates device memory only inside batch-graph and server handles.
 *   - All functions are reentrant; a handle (cs_graph, cs_server) is single-owner.
 */
#ifndef CSIEVE_H
#define CSIEVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cs_status;
#define CS_OK        0
#define CS_EINVAL  (-1)  /* a parameter violates the validation rules below */
#define CS_ERANGE  (-2)  /* a size exceeds a documented limit, or a buffer/workspace is too small */
#define CS_ENOMEM  (-3)  /* host or device allocation failed (handles only) */
#define CS_EDEVICE (-4)  /* a HIP runtime error, or the device reported an internal check */
#define CS_EBUSY   (-5)  /* server: not enough budget or slots now; retry later */

/* One sieve job.  Validation rules (CS_EINVAL unless noted):
 *   2 <= P < 2^24;  d >= 1 squarefree with every prime factor <= P (d | P#);
 *   m_start >= 1;  1 <= m_inc < 2^32;  m_start + m_inc < 2^63;
 *   1 <= sl < 2^17 (a packed row fits an LDS tile) and sl < m_start*K (every N + X > 0);
 *   2 <= limit and max(limit, P) < 2^63 (CS_ERANGE otherwise); primes from 2^42 take the exact
 *   64-bit residue path (Section 3.3: p < 2^64), and limits whose tables exceed device memory go
 *   through the chunked sieve.  Batches, the server and cs_primes take limits below 2^42.
 * A job whose range holds no m coprime to d is valid and has no rows. */
typedef struct cs_job {
  uint32_t P;
  uint32_t sl;
  uint64_t d;
  uint64_t m_start;
  uint64_t m_inc;
  uint64_t limit;
} cs_job;

/* Large-prime enumeration variants; both give identical outputs. */
#define CS_LARGE_G         0u  /* one solve of Eq. 3 by the recursion of Eq. 5 per hit (Section 3.3) */
#define CS_LARGE_THREE_GAP 1u  /* Eq. 5 solves for the first hit and the two return times; then O(1) per hit */

/* Tuning knobs.  Pass NULL for automatic choices.  Outputs never depend on them. */
typedef struct cs_tune {
  uint64_t thr;            /* primes p <= thr take the small-prime branch (Section 5: p/S < C_mult);
                              0 = automatic.  Raised to max(P, 2*sl) (CS_LARGE_G) or 4*sl + 1
                              (CS_LARGE_THREE_GAP) so that each large prime hits a row at most once. */
  uint32_t tile_rows;      /* rows per LDS tile of the small branch; 0 = automatic */
  uint32_t hits_per_item;  /* target expected hits per large-branch work item; 0 = automatic */
  uint32_t large_mode;     /* CS_LARGE_G or CS_LARGE_THREE_GAP */
  uint32_t large_blocks;   /* workgroups of the large branch's grid (each lane takes items with a
                              grid stride); 0 = automatic (128 per CU, 8 per CU with LIST) */
  uint32_t small_slices;   /* prime slices per small-branch tile; 0 = automatic */
  uint32_t branches;       /* cs_sieve_range only: CS_BRANCH_ALL (0), CS_BRANCH_SMALL or
                              CS_BRANCH_LARGE, to run one branch per call (e.g. to time it) */
  uint32_t scatter;        /* how large-prime hits reach the bitmap: CS_SCATTER_AUTO (0),
                              CS_SCATTER_ATOMIC, CS_SCATTER_BYTES or CS_SCATTER_LIST */
  uint32_t list_chunks;    /* CS_SCATTER_LIST: pool capacity in chunks of 4096 hits; 0 = automatic
                              (a smaller pool only moves hits to the atomic fallback) */
  uint32_t walk;           /* which m the large branch visits: CS_WALK_CLASSES (0) only the residue
                              classes of m that can hold rows (odd m when d is even; with one solve
                              per hit m = 1, 5 mod 6 when 6 | d), CS_WALK_ALL every m of the range as
                              the paper's program does (Section 3.2: its solve count then follows
                              the estimate M S (log log limit - log log thr) + pi(limit) - pi(thr)) */
  uint32_t wide_log2;      /* primes p >= 2^wide_log2 take the exact 64-bit residue arithmetic
                              (Montgomery products, integer quotients); 0 = 42, the bound of the
                              fp64 arithmetic; 20..42 move smaller primes onto it (e.g. to check it) */
  uint32_t kmod;           /* where the large branch takes K mod p and m_start K mod p (Eq. 1) from:
                              CS_KMOD_AUTO (0) forms them in the large-branch kernel itself for a
                              single job whose primes all stay below 2^42 (the table then covers only
                              the primes <= thr, for the small branch), else a table built during
                              preparation; CS_KMOD_TABLE (1) always the table.  Outputs are identical. */
} cs_tune;

#define CS_KMOD_AUTO  0u
#define CS_KMOD_TABLE 1u

#define CS_WALK_CLASSES 0u
#define CS_WALK_ALL     1u

/* Large-prime hit scatter.  ATOMIC: per hit, a device-scope atomic OR into the packed bitmap and
 * an atomic add into the row's count.  BYTES: per hit, one atomic add into a byte counter per
 * (row, column) in the workspace (n_m * row_words * 32 bytes, included in cs_layout.ws_bytes);
 * one coalesced pass after the branch ORs the nonzero counters into the bitmap, adds their sums
 * to the counts and clears them.  BYTES is exact only while no number m K + X of the interval can
 * have 256 distinct prime factors above the threshold, i.e. while
 * floor(log2((m_start + m_inc + 1) K) / log2(thr + 1)) < 256; requesting it otherwise gives
 * CS_EINVAL.  LIST: no atomic per hit: each wavefront appends its hits as 32-bit cells
 * (row << s | column, 2^s >= n_x) to a chunk of a workspace pool with coalesced stores; after the
 * branch the cells are grouped by buckets of rows in two counting-sort passes and applied through
 * LDS tiles.  The pool holds about
 * 1.15x the expected number of large hits (n_m n_x (log log limit - log log thr), Mertens); hits
 * beyond it fall back to the atomic path, so results stay exact.  LIST needs n_m * 2^s <= 2^32 and
 * at most 8192 row buckets (CS_EINVAL when requested otherwise).  AUTO, for cs_sieve / cs_prepare
 * / cs_sieve_range: BYTES where exact, else ATOMIC.  Batches use BYTES when every job can, else
 * ATOMIC (they ignore LIST); the server gives each job byte counters where they are exact and
 * its tables with them take at most a quarter of the budget, and an iteration uses BYTES when
 * every job in it has them, else ATOMIC (LIST and an explicit BYTES act as AUTO there; ATOMIC
 * keeps ATOMIC).  With BYTES, a whole-range call runs the
 * small-prime branch on a second stream beside the large one (the large branch writes only its
 * counters until the fold), joined back into `stream` before the call's last kernel.  Outputs are
 * identical in every mode. */
#define CS_SCATTER_AUTO   0u
#define CS_SCATTER_ATOMIC 1u
#define CS_SCATTER_BYTES  2u
#define CS_SCATTER_LIST   3u

#define CS_BRANCH_ALL   0u
#define CS_BRANCH_SMALL 1u
#define CS_BRANCH_LARGE 2u

typedef struct cs_layout {
  uint64_t n_m;            /* rows */
  uint32_t n_x;            /* columns */
  uint32_t row_words;      /* ceil(n_x / 32) */
  uint64_t bitmap_bytes;   /* n_m * row_words * 4 */
  uint64_t counts_bytes;   /* n_m * 4 */
  uint64_t ws_bytes;       /* device workspace needed by cs_sieve / cs_prepare / cs_sieve_range */
  uint64_t prime_cap;      /* capacity of the prime table: an upper bound of pi(max(limit, P)) */
  uint64_t thr;            /* effective small/large threshold for the given tuning */
  uint32_t scatter;        /* large-hit scatter cs_sieve uses: CS_SCATTER_ATOMIC, _BYTES or _LIST */
  uint32_t reserved;
} cs_layout;

/* Prime decades of the per-decade counters: decade i holds the primes 10^i <= p < 10^(i+1). */
#define CS_DECADES 20

/* Counters accumulated by the kernels of the last cs_prepare + cs_sieve_range calls on a
 * workspace (cs_sieve resets them).  small_primes / large_primes count the primes of the branches
 * each call ran (cs_tune.branches), so a SMALL call and a LARGE call over the same range count
 * every prime once.  The dec_* arrays split the large branch's counters by prime decade; each
 * total above equals the sum of its array. */
typedef struct cs_diag {
  uint64_t n_primes;        /* primes <= max(limit, P) in the table */
  uint64_t small_primes;    /* primes handed to the small branch */
  uint64_t large_primes;    /* primes handed to the large branch */
  uint64_t small_pairs;     /* (row, prime) residues N mod p computed by the small branch */
  uint64_t small_marks;     /* column marks (= factors) added by the small branch */
  uint64_t large_raw_hits;  /* solutions (m, X) of Eq. 3 found, any m in range, any X */
  uint64_t large_hits;      /* ... with gcd(m, d) = 1 and X a column (= factors added) */
  uint64_t g_calls;         /* solves of Eq. 3 by the recursion of Eq. 5 */
  uint64_t g_levels;        /* recursion levels summed over those solves */
  uint64_t error_flags;     /* nonzero: a device-side consistency check failed */
  double large_kernel_ms;   /* duration of the last large-branch kernel launched on this workspace
                               (HIP events on its stream; 0 if none, or launched under capture) */
  uint64_t dec_primes[CS_DECADES];    /* large primes per decade (= large_primes in total) */
  uint64_t dec_raw_hits[CS_DECADES];  /* large_raw_hits per decade of the prime */
  uint64_t dec_hits[CS_DECADES];      /* large_hits per decade */
  uint64_t dec_solves[CS_DECADES];    /* g_calls per decade */
  uint64_t dec_levels[CS_DECADES];    /* g_levels per decade */
} cs_diag;

/* Human-readable name of a status code (static string). */
const char* cs_strerror(cs_status st);

/* Text of the last HIP runtime failure seen by this thread's calls ("kernel: message"), or ""
 * if none.  Static thread-local storage; valid until the thread's next failing call. */
const char* cs_last_error(void);

/* Validates `job` and fills `out` (host only, no device work).  `tune` may be NULL. */
cs_status cs_plan(const cs_job* job, const cs_tune* tune, cs_layout* out);

/* Host only.  Column c -> X, for c < min(cap, n_x).  Errors: CS_EINVAL (invalid job). */
cs_status cs_columns(const cs_job* job, int32_t* x_of_col, uint64_t cap);

/* Host only.  Row r -> m, for r < min(cap, n_m). */
cs_status cs_rows(const cs_job* job, uint64_t* m_of_row, uint64_t cap);

/* The whole sieve (Sections 3.1-3.3): clears d_bitmap and d_counts, builds the prime table
 * up to max(limit, P), K mod p for every prime (Eq. 1 cache), then runs the small-prime
 * branch (primes <= thr, marked in LDS tiles of rows) and the large-prime branch (primes
 * > thr, Eq. 3 solved by Eq. 5; hits reach the bitmap by the scatter of cs_tune.scatter).
 * With byte counters the small branch runs on a second, library-owned stream beside the large
 * one (joined back before the call's last launch; not under graph capture).
 * d_bitmap: layout.bitmap_bytes; d_counts: layout.counts_bytes; d_ws: layout.ws_bytes
 * (CS_ERANGE if ws_bytes is smaller).  All three are caller-owned device memory. */
cs_status cs_sieve(const cs_job* job, const cs_tune* tune, uint32_t* d_bitmap, uint32_t* d_counts,
                   void* d_ws, uint64_t ws_bytes, void* stream);

/* cs_sieve for callers that cannot allocate device memory (code under graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same sieve, with the workspace taken from
 * a device array the library holds, cs_scratch_bytes() = 256 MiB, one per device (allocated when
 * the library's code object is loaded on that device and held until the process ends).  Jobs
 * whose cs_plan ws_bytes exceed it get CS_ERANGE (nothing enqueued).  Everything runs on `stream`
 * (no second stream, no timing events: cs_diag.large_kernel_ms is not updated).  The call allocates
 * nothing.  Every call on a device shares that device's array, which keeps the last call's
 * contents (each call clears what must start at zero): calls that overlap on one device race, so
 * the caller serialises them (one stream, or events between streams).  The diagnostic counters
 * live in that array too and are not readable through cs_diag_read. */
cs_status cs_sieve_noalloc(const cs_job* job, const cs_tune* tune, uint32_t* d_bitmap, uint32_t* d_counts,
                           void* stream);
uint64_t cs_scratch_bytes(void);

/* First half of cs_sieve without touching any output: prime table, K mod p, row and column
 * tables into d_ws, and the diagnostic counters reset. */
cs_status cs_prepare(const cs_job* job, const cs_tune* tune, void* d_ws, uint64_t ws_bytes,
                     void* stream);

/* Sieves with the primes p in [p_lo, p_hi] only (clipped to [2, limit]) and ORs the marks
 * into d_bitmap and adds the factors into d_counts.  d_ws must hold the tables of the same
 * job and tuning from cs_prepare, earlier on the same stream.  Splitting [2, limit] into
 * ranges and calling this once per range gives exactly cs_sieve's result (bitwise OR and
 * integer sums are order independent), which makes a job splittable and resumable. */
cs_status cs_sieve_range(const cs_job* job, const cs_tune* tune, uint64_t p_lo, uint64_t p_hi,
                         uint32_t* d_bitmap, uint32_t* d_counts, void* d_ws, uint64_t ws_bytes,
                         void* stream);

/* The whole sieve with the prime range taken in chunks of `span` integers: for each chunk
 * [a, a + span) in turn, its primes (the segmented sieve restarted at a), their K mod p (Eq. 1),
 * then both branches over them, exactly as cs_sieve_range with [a, a + span - 1].  Only one
 * chunk's prime, K mod p and m_start*K mod p tables (24 bytes a prime) are held, so limits whose
 * tables would exceed device memory fit (Section 3.1's space-time tradeoff, applied per chunk).
 * The result is exactly cs_sieve's.  span: a multiple of 2^19, at least 2^25 and above P
 * (CS_EINVAL otherwise); span > limit is the unchunked sieve.  d_ws: cs_plan_chunked's
 * ws_bytes for the same span (CS_ERANGE if smaller); layout.prime_cap is then the capacity of
 * one chunk's table (a chunk with more primes than [0, span) sets error_flags' prime-table bit,
 * reported by cs_diag_read).  cs_diag's large_kernel_ms covers the last chunk's launch. */
cs_status cs_plan_chunked(const cs_job* job, const cs_tune* tune, uint64_t span, cs_layout* out);
cs_status cs_sieve_chunked(const cs_job* job, const cs_tune* tune, uint64_t span, uint32_t* d_bitmap,
                           uint32_t* d_counts, void* d_ws, uint64_t ws_bytes, void* stream);

/* The chunked sieve restricted to the primes p in [p_lo, p_hi] (clipped to [2, limit]): ORs their
 * marks into d_bitmap and adds their factors into d_counts (nothing is cleared), like
 * cs_sieve_range, with the chunks of the prime range that hold no such prime skipped (the first
 * chunk is always prepared: it supplies K's prime groups and the row and column tables).
 * Splitting [2, limit] into ranges gives exactly cs_sieve_chunked's result. */
cs_status cs_sieve_chunked_range(const cs_job* job, const cs_tune* tune, uint64_t span, uint64_t p_lo,
                                 uint64_t p_hi, uint32_t* d_bitmap, uint32_t* d_counts, void* d_ws,
                                 uint64_t ws_bytes, void* stream);

/* Waits for `stream`, then copies the counters kept in d_ws (see cs_diag).  Returns
 * CS_EDEVICE if the stream reported an error or error_flags is nonzero. */
cs_status cs_diag_read(const void* d_ws, cs_diag* out, void* stream);

/* Prime table alone (the segmented sieve of Eratosthenes behind cs_sieve; the paper counts
 * it as a one-time cost, Section 5): writes the primes <= limit ascending to d_primes
 * (capacity `cap`, CS_ERANGE if smaller than cs_primes_ws's *cap_out) and their number to
 * *d_count (device uint64).  ws: cs_primes_ws bytes. */
cs_status cs_primes_ws(uint64_t limit, uint64_t* cap_out, uint64_t* ws_bytes_out);
cs_status cs_primes(uint64_t limit, uint64_t* d_primes, uint64_t cap, uint64_t* d_count,
                    void* d_ws, uint64_t ws_bytes, void* stream);

/* K mod p for n primes (Eq. 1: the cached residue, K = P#/d): d_out[i] = K mod d_primes[i].
 * Every d_primes[i] must be a prime below 2^63 (from 2^42 on the products are exact 64-bit
 * Montgomery products).  d_ws: cs_kmod_ws bytes (it receives the
 * products of the primes dividing K, grouped below 2^50). */
cs_status cs_kmod_ws(uint32_t P, uint64_t d, uint64_t* ws_bytes_out);
cs_status cs_kmod(uint32_t P, uint64_t d, const uint64_t* d_primes, uint64_t n, uint64_t* d_out,
                  void* d_ws, uint64_t ws_bytes, void* stream);

/* Scatter-rate probe (measurement only, not part of the sieve): n_ops 32-bit operations at
 * pseudo-random words of d_buf (words uint32, device memory), the words drawn from a 64-bit mixing
 * hash of the operation index and `seed` in registers, so that the probe loads no indices.
 * op 0: atomic add of 1 at device scope (the byte-counter and atomic scatters' operation);
 * op 1: plain 4-byte store of a nonzero value; op 2: atomic add of 1 into a 64 KB LDS table per
 * workgroup (the LDS-tile scatters' operation; only the op count reaches d_buf[0]).
 * slices > 1 (at most 16): the buffer is cut into `slices` equal ranges and each workgroup uses
 * only the range of its XCD (hardware id mod slices).  After op 0 the words sum to n_ops (plus
 * their previous contents).  Errors: CS_EINVAL (null buffer, op > 2, slices 0 or > 16, fewer
 * words than slices).  Enqueued on `stream`; the caller times it (e.g. with events). */
cs_status cs_probe_scatter(uint32_t* d_buf, uint64_t words, uint64_t n_ops, uint32_t slices, uint32_t op,
                           uint64_t seed, void* stream);

/* ------------------------------------------------------------------------------------------
 * Probable-prime stage (after the sieve).  Section 2 ("Larger Gaps", "Sieving"): the numbers
 * of an interval that the sieve left unmarked are tested for primality walking away from N on
 * both sides until the surrounding primes are found; their distance is the gap containing N and
 * gap / log(lower prime) its merit (Section 1).  Section 2.2: the test is probabilistic; the
 * one here is the strong probable-prime test to base 2 (the first half of BPSW): with
 * n - 1 = 2^s t, t odd, n passes iff 2^t = 1 or 2^(2^r t) = -1 (mod n) for some 0 <= r < s.
 * Primes always pass; so do the (rare) strong pseudoprimes to base 2, e.g. 2047 = 23 * 89.
 * ------------------------------------------------------------------------------------------ */

/* The test for n numbers of n_limbs 32-bit limbs each (little endian; number i at
 * d_limbs + i * n_limbs): d_out[i] = 1 if it passes, else 0 (also for 0, 1 and even numbers
 * other than 2).  1 <= n_limbs <= 64 (numbers below 2^2048), CS_ERANGE otherwise.  Device
 * buffers; enqueued on `stream`, no workspace. */
cs_status cs_prp_numbers(const uint32_t* d_limbs, uint32_t n_limbs, uint64_t n, uint8_t* d_out, void* stream);

/* The tests of BPSW (Section 2.2: the paper's search tests with GMP's probable-prime routine, a
 * BPSW test).  CS_PRP_SPRP2 is the strong test to base 2 above.  CS_PRP_LUCAS is the strong Lucas
 * test with Selfridge's parameters: D the first of 5, -7, 9, -11, ... with Jacobi symbol
 * (D/n) = -1, P = 1, Q = (1 - D)/4; with n + 1 = 2^s d, d odd, n passes iff U_d = 0 or
 * V_(2^r d) = 0 (mod n) for some 0 <= r < s, where U, V are the Lucas sequences of (P, Q).  Even
 * n other than 2, 0, 1, perfect squares and n with (D/n) = 0 for some |D| != n before a D with
 * (D/n) = -1 fail.  (Under the generalised Riemann hypothesis every other n < 2^2048 has such a
 * D below 2^23; a search reaching 2^23 reports n composite, and a perfect square of 2^32 or more
 * is found composite that way, after about 4 million Jacobi symbols.)  CS_PRP_BPSW: both (the
 * Lucas test only for numbers passing the first); no composite is known to pass. */
#define CS_PRP_SPRP2 0u
#define CS_PRP_LUCAS 1u
#define CS_PRP_BPSW  2u

/* cs_prp_numbers with a choice of test (CS_PRP_*; CS_EINVAL for another value); same buffers,
 * limits and errors.  The Lucas and BPSW tests take a quad of lanes per number. */
cs_status cs_prp_test(const uint32_t* d_limbs, uint32_t n_limbs, uint64_t n, uint32_t test, uint8_t* d_out,
                      void* stream);

/* Result of the surrounding-prime search for one row, N = m*K. */
typedef struct cs_surround_row {
  int32_t prev;         /* largest X < 0 with N + X a BPSW probable prime, searched among the
                           unmarked columns in [-sl, -1]; 0 if there is none */
  int32_t next;         /* smallest such X > 0 in [1, sl]; 0 if none */
  uint32_t tests_prev;  /* unmarked columns on that side up to and including prev (all of them
                           when prev = 0): the strong tests to base 2 a sequential search runs */
  uint32_t tests_next;
} cs_surround_row;

typedef struct cs_surround_stats {
  uint64_t rounds;      /* gather/test/resolve rounds run */
  uint64_t tests;       /* tests run, including those past a side's first probable prime */
  uint64_t limbs;       /* 32-bit limbs per number in the test kernel */
  uint64_t bits;        /* bit length of K plus that of the largest m: every N + X tested has
                           this many bits or one fewer (one more only if X > 0 carries) */
  double test_ms;       /* time of the test kernels alone (HIP events on `stream`) */
  uint64_t lucas_tests; /* strong Lucas tests run: every pass tests each side that holds a
                           probable prime */
  uint64_t lucas_passes;/* passes of the Lucas test over the sides (more than one only when a
                           strong pseudoprime to base 2 was found and its side searched on) */
  double lucas_ms;      /* time of the Lucas passes (HIP events on `stream`) */
} cs_surround_stats;

/* Workspace bytes of cs_surround for n_rows rows of this job (host only). */
cs_status cs_surround_ws(const cs_job* job, uint64_t n_rows, uint64_t* ws_bytes);

/* Surrounding probable primes of n_rows rows of a sieved job: the nearest BPSW probable primes on
 * both sides of N = m K.
 * d_bitmap: n_rows rows of row_words words in cs_sieve's layout (1 = marked composite), the
 * rows to search (e.g. a slice of cs_sieve's bitmap); d_m[i]: the m of row i, within
 * [m_start, m_start + m_inc) (a device-side check reports CS_EDEVICE otherwise); d_out: n_rows
 * results.  Candidates per side are tested with the strong test to base 2 in rounds of up to
 * 1024 at once and the first probable prime in walking order is kept; the strong Lucas test then
 * checks each side's number, and a side whose number fails searches on past it, so results equal
 * a sequential BPSW search's.
 * N = m K + sl must stay below 2^2048 (CS_ERANGE).  Synchronous: returns after the work has
 * completed (one host read of a counter per round).  stats may be NULL. */
cs_status cs_surround(const cs_job* job, const uint32_t* d_bitmap, const uint64_t* d_m, uint64_t n_rows,
                      cs_surround_row* d_out, void* d_ws, uint64_t ws_bytes, cs_surround_stats* stats,
                      void* stream);

/* ------------------------------------------------------------------------------------------
 * Batches: many jobs (different P, d, m ranges, sl, limits) sieved by one sequence of fused
 * launches.  The prime table is built once up to the largest limit and shared; the per-job
 * preparation kernels each cover every job in a single launch.  The sieve branches then run on
 * one of two paths:
 *   CS_BATCH_PERSISTENT  one launch of a persistent kernel whose workgroups pop tasks from a
 *                        device queue until it is empty: every job's large-branch items in tasks
 *                        of 1024, then every job's small-branch units; the byte counters of all
 *                        jobs are folded by one fused launch after it.  Needs one large-prime
 *                        enumeration (cs_tune.large_mode) for all jobs and every job's column
 *                        table plus one tile row within 40 KB of LDS (sl up to about 40,000).
 *   CS_BATCH_LANES       each job's branches as single-job launches spread over lane streams
 *                        that fork from and join the caller's stream.
 * A batch handle captures its sequence once in a hipGraph and replays it.  Outputs are
 * bit-identical to one cs_sieve call per job on either path.
 * ------------------------------------------------------------------------------------------ */
typedef struct cs_batch cs_batch;

#define CS_BATCH_AUTO       0u   /* persistent when the jobs admit it, else lanes */
#define CS_BATCH_PERSISTENT 1u
#define CS_BATCH_LANES      2u

#define CS_ORDER_AUTO        0u  /* persistent task queue order: CS_ORDER_BY_JOB */
#define CS_ORDER_LARGE_FIRST 1u  /* every job's large tasks, then every job's small ones */
#define CS_ORDER_SMALL_FIRST 2u
#define CS_ORDER_BY_JOB      3u  /* job by job, each job's large tasks then its small ones */

/* Batch-level knobs (outputs never depend on them).  NULL = all zero = automatic. */
typedef struct cs_batch_opts {
  uint32_t path;            /* CS_BATCH_AUTO, CS_BATCH_PERSISTENT or CS_BATCH_LANES */
  uint32_t items_per_task;  /* persistent: large-branch work items (prime x m-chunk) per task, a
                               multiple of 256 up to 8192; 0 = 1024 */
  uint32_t blocks_per_cu;   /* persistent: workgroups per CU (1-8); 0 = 4 */
  uint32_t order;           /* persistent: CS_ORDER_* of the task queue */
} cs_batch_opts;

/* Validates and plans every job, allocates the batch's device memory (prime table, per-job
 * tables; see cs_batch_layout's ws_bytes) on the current device.  tunes: n entries or NULL;
 * opts may be NULL (cs_batch_create passes NULL).  Errors: those of cs_plan for any job;
 * CS_EINVAL for CS_BATCH_PERSISTENT when the jobs do not admit it, or knobs out of range;
 * CS_ENOMEM; CS_EDEVICE. */
cs_status cs_batch_create(const cs_job* jobs, uint32_t n, const cs_tune* tunes, cs_batch** out);
cs_status cs_batch_create_ex(const cs_job* jobs, uint32_t n, const cs_tune* tunes, const cs_batch_opts* opts,
                             cs_batch** out);

/* The path a handle runs: CS_BATCH_PERSISTENT or CS_BATCH_LANES (0 for NULL). */
uint32_t cs_batch_path(const cs_batch* b);

/* The whole batch in one call on the caller's stream and workspace (nothing allocated, no
 * graph, no second stream): the persistent path when the jobs admit it, else each job's branch
 * launches in turn on `stream`.  cs_batch_ws gives the workspace bytes (host only).  d_bitmaps /
 * d_counts: n caller-owned outputs in cs_sieve's layout (NULL allowed for jobs without rows).
 * Errors: those of cs_plan for any job; CS_ERANGE if ws_bytes is too small. */
cs_status cs_batch_ws(const cs_job* jobs, uint32_t n, const cs_tune* tunes, uint64_t* ws_bytes);
cs_status cs_sieve_batch(const cs_job* jobs, uint32_t n, const cs_tune* tunes, const cs_batch_opts* opts,
                         uint32_t* const* d_bitmaps, uint32_t* const* d_counts, void* d_ws, uint64_t ws_bytes,
                         void* stream);

/* Layout of job i (n_m, n_x, row_words, bitmap and counts bytes); ws_bytes is the batch's
 * total device memory. */
cs_status cs_batch_layout(const cs_batch* b, uint32_t i, cs_layout* out);

/* Sieves every job into its caller-owned outputs d_bitmaps[i] / d_counts[i] (sizes from
 * cs_batch_layout), on `stream`.  use_graph != 0: the launch sequence is captured into a
 * hipGraph on the first call (and again whenever the output pointers change) and replayed;
 * use_graph = 0: the same launches are enqueued directly.  Calls on one handle must not
 * overlap on the device (they share the handle's tables). */
cs_status cs_batch_run(cs_batch* b, uint32_t* const* d_bitmaps, uint32_t* const* d_counts,
                       int use_graph, void* stream);

/* Waits for `stream` and reads the batch's counters (summed over jobs). */
cs_status cs_batch_diag(cs_batch* b, cs_diag* out, void* stream);

/* Frees the handle (waits for the device first).  NULL is a no-op. */
cs_status cs_batch_destroy(cs_batch* b);

/* ------------------------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.  The server keeps the prime table (up to
 * max_limit) and K mod p tables (per (P, d), reused by any later job whose limit they cover)
 * resident, admits queued jobs in arrival order as slots and budget allow, and runs
 * iterations on its own stream: one iteration is one fused launch sequence that advances every
 * active job by one prime-range chunk (`chunks` ranges of large primes of about equal prime
 * count, the first of them together with the small primes, whose branch runs on a second stream
 * beside the large one).  Jobs that arrive while others run join the next iteration.  Each job's result is
 * bit-identical to cs_sieve of that job alone.  Outputs live in the server's memory until
 * released.  A server handle may be used from several host threads.
 * ------------------------------------------------------------------------------------------ */
typedef struct cs_server cs_server;

typedef struct cs_server_config {
  uint64_t budget_bytes;   /* device bytes for per-job tables, K mod p tables and outputs */
  uint64_t max_limit;      /* largest max(limit, P) accepted; the resident prime table reaches it */
  uint32_t max_active;     /* jobs in flight at once (slots) */
  uint32_t chunks;         /* large-prime chunks per job, one per iteration (0 = 1: every job in one
                              iteration, measured best for latency on mixed jobs) */
  cs_tune tune;            /* applied to every job; with thr = 0 and CS_LARGE_THREE_GAP each job's
                              threshold is 44 n_x (the small and large branches of many jobs share
                              the device at once, so their costs add: n_m 1.25 ps per small prime
                              against n_m n_x / p hit atomics of 55 ps per large one) */
  double long_ms;          /* > 0: jobs whose estimated device time alone exceeds this many ms run
                              in a second lane (its own loop, streams and iterations) beside the
                              others, so that their iterations do not wait for the long jobs;
                              0: one lane.  The estimate (from the plan: the large branch's hits
                              by Mertens' theorem and its per-prime setup, and the small branch's
                              pairs) changes no result. */
} cs_server_config;

typedef struct cs_ticket_info {
  int32_t state;           /* 0 queued, 1 running, 2 done, -1 failed */
  uint32_t n_x;
  uint32_t row_words;
  uint32_t pad;
  uint64_t n_m;
  double queued_s;         /* submit -> admission (or now) */
  double latency_s;        /* submit -> completion (or now) */
} cs_ticket_info;

typedef struct cs_server_stats {
  uint64_t submitted, admitted, completed, failed, iterations;
  uint64_t kmod_builds, kmod_hits, kmod_evictions;
  uint64_t bytes_in_use, active, queued;
  uint64_t bytes_iterations;   /* iterations whose large branch used the byte counters */
} cs_server_counters;

/* Allocates budget_bytes plus the prime table on the current device, builds the prime table
 * and starts the server thread.  Errors: CS_EINVAL, CS_ERANGE (max_limit), CS_ENOMEM,
 * CS_EDEVICE. */
cs_status cs_server_create(const cs_server_config* cfg, cs_server** out);

/* Queues a job and returns its ticket; never blocks on the device.  CS_ERANGE if the job can
 * never fit the budget or its limit exceeds max_limit; validation errors as cs_plan. */
cs_status cs_server_submit(cs_server* s, const cs_job* job, uint64_t* ticket);

/* State and timing of a ticket (CS_EDEVICE if it failed). */
cs_status cs_server_poll(cs_server* s, uint64_t ticket, cs_ticket_info* out);

/* Waits until the ticket is done or failed, at most timeout_s seconds (CS_EBUSY on timeout). */
cs_status cs_server_wait(cs_server* s, uint64_t ticket, double timeout_s, cs_ticket_info* out);

/* Copies a done ticket's outputs (layout as cs_sieve) to caller-owned device buffers on
 * `stream`.  CS_EBUSY if not done yet. */
cs_status cs_server_copy_outputs(cs_server* s, uint64_t ticket, uint32_t* d_bitmap, uint32_t* d_counts,
                                 void* stream);

/* Frees a finished ticket's outputs (synchronise any copy first).  CS_EBUSY if still running. */
cs_status cs_server_release(cs_server* s, uint64_t ticket);

cs_status cs_server_stats(cs_server* s, cs_server_counters* out);

/* Stops the thread after the current iteration and frees everything.  NULL is a no-op. */
cs_status cs_server_destroy(cs_server* s);

#ifdef __cplusplus
}
#endif

#endif /* CSIEVE_H */

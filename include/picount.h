/*
 * picount.h -- C ABI of the MI355X (gfx950) prime-counting library.
 *
 * The library computes pi(x), the number of primes <= x (Section 1 of
 * D. B. Staple, "The combinatorial algorithm for computing pi(x)",
 * arXiv:1503.01839), by the combinatorial method:
 *
 *   pi(x) = phi(x, a) + a - 1 - P2(x, a),    a = pi(y),  icbrt(x) <= y <= isqrt(x)
 *   phi(x, a) = S1 + S2                     (the tree of eq. (4.1), Section 4)
 *
 * phi(u, b) counts the naturals <= u coprime to the first b primes
 * (Section 3).  S1 sums the ordinary leaves, S2 the special leaves
 * -mu(m) phi(x/(m p_b), b-1) over c < b < a, m squarefree with lpf(m) > p_b
 * and y/p_b < m <= y; c is the wheel size (Section 4).  Special leaves are
 * trivial (u = x/(m p_b) < p_b), easy (p_b <= u < p_b^2, u <= y: Legendre's
 * formula, Section 4) or hard (every other leaf: phi read from a segmented
 * sieve of [1, x/y] with per-prime running counts, Sections 2.3 and 3).
 * P2 counts n = p q <= x with p_a < p <= q.
 *
 * Every step runs in hand-written HIP kernels on the current HIP device; the
 * host only plans, launches and reads back a few 128-bit partial sums.
 *
 * Conventions for every entry point:
 *  - Returns PC_OK or an error status; outputs are written only on PC_OK.
 *  - Pointer arguments named *_out / out are host pointers owned by the
 *    caller; the library never frees caller memory.
 *  - Calls are synchronous unless named *_async.  The library keeps shared
 *    read-only tables (primes, pi, mu*lpf) on the device between calls and
 *    grows them on demand; pc_shutdown() releases them.
 *  - Calls from several host threads are serialised internally.
 *  - On error, pc_last_error() (thread-local) describes the failure.
 */
#ifndef PICOUNT_H
#define PICOUNT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PC_OK = 0,
    PC_EINVAL = 1,    /* an argument is outside its documented domain      */
    PC_ERANGE = 2,    /* x or a derived size exceeds what the build handles */
    PC_ENOMEM = 3,    /* device memory or a caller workspace is too small   */
    PC_EDEVICE = 4,   /* a HIP runtime call failed                          */
    PC_EINTERNAL = 5  /* an internal consistency check failed               */
} pc_status;

/* Signed 128-bit integer: value = hi * 2^64 + lo. */
typedef struct {
    uint64_t lo;
    int64_t hi;
} pc_i128;

/* Tuning knobs.  Zero in any field means "library default". */
typedef struct {
    double alpha;          /* y = alpha * icbrt(x), clamped to [icbrt x, isqrt x]; 0 = tuned */
    uint32_t segment_kib;  /* LDS bitmap per sieve segment: 32 or 64                       */
    uint32_t wg_size;      /* sieve workgroup: 256|512 (32 KiB segments), 512|1024 (64)   */
    uint32_t tile_leaves;  /* leaf items per sieve tile (hot segments split by columns); 0 = 2^22, 0xFFFFFFFF = off */
    uint32_t flags;        /* PC_FLAG_* below */
    uint64_t carry_budget; /* bytes for per-(segment, prime) counts per window; 0 = auto  */
    uint32_t small_span;   /* one-wavefront segments cover [0, small_span * y); 0 = none    */
    uint32_t small_kib;    /* size of those segments: 4 or 8 KiB; 0 = auto                  */
} pc_config;

#define PC_FLAG_TWO_PASS 1u      /* count pass, carry scan, then leaf pass (else one tally pass) */
#define PC_FLAG_NO_BATCH_LARGE 2u /* cross large primes one at a time (no batched crossing)     */
#define PC_FLAG_REBUILD_TABLES 4u /* rebuild the cached tables inside this call (into the same
                                     device memory; pc_shutdown frees it)                        */
#define PC_FLAG_NO_SMALL_SEGMENTS 8u /* no one-wavefront segments even if small_span is set        */
#define PC_FLAG_NO_GRAPH 16u         /* batches: launch each phase directly, not as a HIP graph     */
#define PC_FLAG_BATCH_SEQUENTIAL 32u /* batches: one query after another (the plain per-query path) */
#define PC_FLAG_SEEDED 64u           /* windows of segments seeded on their own with phi(m_min, b)
                                        (Section 4) instead of carried from the window before;
                                        they then run last to first                               */

/* Everything one pi(x) evaluation produced, for tests and measurement. */
typedef struct {
    uint64_t x, y, a, c, z, bmax;   /* parameters actually used                     */
    uint64_t pi;                    /* pi(x)                                        */
    pc_i128 s1, s2_trivial, s2_easy, s2_hard, p2, phi; /* phi = S1 + S2          */
    uint64_t n_s1, n_trivial, n_easy, n_hard, n_p2;    /* term / leaf counts       */
    uint64_t segments, tiles, windows;
    uint64_t segment_bits;          /* bits (odd integers) per workgroup segment     */
    uint64_t small_segments;        /* leading one-wavefront segments (of the total) */
    uint64_t crossings;             /* odd multiples of p_{c+1}..p_bmax below the sieve end */
    uint64_t device_bytes;          /* peak device bytes held by the library        */
    uint32_t sieve_launches, scan_launches;
    /* ms_total, ms_tables, ms_sieve: host wall clock of the call, of the table
     * build and from the sieve's start to the result.  ms_leaves: GPU time from
     * the start of S1 to the end of the easy leaves, which run on a second
     * stream concurrently with the sieve. */
    double ms_total, ms_tables, ms_leaves, ms_sieve;
    double ms_k_sieve, ms_k_scan, ms_k_easy, ms_k_s1;  /* kernel time, HIP events     */
    uint64_t n_easy_items;          /* work items of the easy-leaf kernels: a candidate m,
                                       a single prime m, or a value K = pi(u) of a run
                                       of primes m sharing it                   */
    uint64_t x_hi;                  /* x = x_hi * 2^64 + x (pc_pi_count_wide)       */
    uint64_t pi_hi;                 /* pi(x) = pi_hi * 2^64 + pi (pc_pi_count_wide) */
    double ms_k_seed;               /* kernel time of the window seeds (PC_FLAG_SEEDED) */
} pc_result;

/* ---------------------------------------------------------------------- */

/* pi(x) for 0 <= x < 2^64 (Section 1).  alpha selects y = alpha*icbrt(x)
 * (Section 2: y_max = alpha x^(1/3)), clamped to [icbrt x, isqrt x]; alpha = 0
 * picks a tuned value; alpha < 0 or NaN -> PC_EINVAL.  pi(0) = pi(1) = 0.
 * Small x (x < 2^20) is answered from the device pi table. */
pc_status pc_pi_count(uint64_t x, double alpha, uint64_t *pi_out);

/* As pc_pi_count with explicit knobs (cfg may be NULL) and the full
 * decomposition in *res (may be NULL). */
pc_status pc_pi_count_ex(uint64_t x, const pc_config *cfg, pc_result *res);

/* pi(x) for x = x_hi * 2^64 + x_lo, 0 <= x <= 2^72 (else PC_ERANGE): the
 * range of Table 2's 2^64 .. 2^72 and Table 1's 10^20 and 10^21 (Section 5).
 * Knobs and *res (either may be NULL) as in pc_pi_count_ex; res->x, res->x_hi
 * hold the two words of x and res->pi, res->pi_hi those of pi(x) (pi(x) passes
 * 2^64 from x = 2^70 on).  Above 2^64 the method is unchanged: every leaf
 * quotient, every x / p of P2 and every segment bound stays below 2^64; X_b,
 * S1's x / n and the sums are taken in 128 bits; the pi table reaches
 * isqrt(x) <= 2^36 with the primes above 2^32 held as 64-bit values (about
 * 54 GB of device memory at 2^72, the stored counts cut into 6 GiB windows). */
pc_status pc_pi_count_wide(uint64_t x_lo, uint64_t x_hi, const pc_config *cfg, pc_result *res);

/* Hard special-leaf sum S2h = -sum over hard leaves of mu(m) phi(u, b-1),
 * u = floor(x/(m p_b)) (Sections 2.3 and 3).  Requires
 * icbrt(x) <= y <= isqrt(x) and a == pi(y), else PC_EINVAL; x >= 8.
 * The wheel size is c = min(pc_wheel_c(), a). */
pc_status pc_s2_hard(uint64_t x, uint64_t y, uint64_t a, pc_i128 *out);

/* As pc_s2_hard with knobs and the full decomposition (S1, S2t, S2e, S2h and
 * P2 are all computed; pi in *res is Meissel's identity with this y). */
pc_status pc_decompose(uint64_t x, uint64_t y, const pc_config *cfg, pc_result *res);

/* P2(x, pi(y)) = #{n <= x : n = p q, y < p <= q} = sum over primes
 * y < p <= sqrt x of (pi(x/p) - pi(p) + 1), with pi(x/p) read from the same
 * segmented sieve of [1, x/y].  Same y validation as pc_s2_hard. */
pc_status pc_p2(uint64_t x, uint64_t y, uint64_t *out);

/* pi(xs[i]) for i < n; host arrays of n elements.  n = 0 is valid.  Every
 * xs[i] is validated before any work; on error nothing is written and
 * pc_last_error() names the first bad index.  All queries share one set of
 * device tables and run in rounds that fit the round budget (6 GiB of sieve
 * counts): per round one set-up pass, one easy-leaf pass, one sieve launch
 * whose (query, segment) tiles cover every query of the round, one carry
 * pass and one combination, captured as a HIP graph.  A query too large for
 * a round runs alone, windowed.  alpha per query comes from the tuning
 * table's batch column (the alpha of least total work for a batch of queries
 * of that size, which may differ from a lone query's). */
pc_status pc_pi_count_batch(const uint64_t *xs, size_t n, uint64_t *pi_out);

/* As pc_pi_count_batch with knobs; cfg may be NULL. */
pc_status pc_pi_count_batch_ex(const uint64_t *xs, size_t n, const pc_config *cfg,
                               uint64_t *pi_out);

/* The batch in caller memory, for callers that own device memory and
 * streams (a framework's allocator and current stream).
 *
 * pc_workspace_bytes: device bytes of workspace that
 * pc_pi_count_batch_async needs for these n queries (host array xs).  The
 * figure covers each round's uploaded arrays (query scalars, block tables
 * and sieve tiles: 16 bytes per segment of every query, a few hundred bytes
 * per query), one round arena (per-segment counts and weights of a round's
 * queries, 8 bytes per segment per sieving prime, bounded by the 6 GiB round
 * budget, plus each query's per-prime arrays) and 16 bytes per query answered
 * on the host.  n = 0 gives 0.  Returns SIZE_MAX on error (xs null with
 * n > 0, a device table that cannot be built); pc_last_error() says why.
 * Builds the shared device tables these queries need, as the other calls do.
 *
 * pc_pi_count_batch_async: d_out[i] = pi(d_xs[i]) for i < n, every step on
 * hip_stream (a hipStream_t; NULL is the null stream).  d_xs, d_out and d_ws
 * are device pointers owned by the caller: d_xs of n elements, d_out of n
 * elements, d_ws of ws_bytes >= pc_workspace_bytes(xs, n) bytes (256-byte
 * aligned, as hipMalloc returns).  The call first waits for the stream's
 * earlier work and reads d_xs back (it plans on the host), so d_xs may be
 * reused once it returns.  Queries whose sieve counts exceed the round
 * budget (x above a few times 10^17 at the tuned alpha) are computed during the call
 * on the library's own stream; everything else is queued on hip_stream and
 * the call returns without waiting for it: d_out is complete once the stream
 * reaches that point, and d_out and d_ws must stay allocated until then.
 * The call queues no allocation and no memset, but it synchronises the
 * stream, so it cannot be captured into a HIP graph.  Too small a workspace
 * gives PC_ENOMEM before anything is queued or written.  d_out[i] is all
 * ones if the device found an internal inconsistency for that query (pi(x) <
 * 2^63 for every x < 2^64, so no count has that value).  n = 0 is valid and
 * touches nothing; d_xs or d_out null with n > 0 gives PC_EINVAL.  The shared
 * tables stay valid for queued batches: a later call that has to grow them
 * first waits for every queued batch. */
size_t pc_workspace_bytes(const uint64_t *xs, size_t n);
pc_status pc_pi_count_batch_async(const uint64_t *d_xs, size_t n, uint64_t *d_out, void *d_ws,
                                  size_t ws_bytes, void *hip_stream);

/* The caller-memory batch without any allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  d_out[i] = pi(d_xs[i]) for i < n, as
 * pc_pi_count_batch_async computes it, with the same device arrays d_xs and
 * d_out (n elements each) and stream; no workspace argument: the workspace is
 * a fixed device array of the library, PC_NOALLOC_SCRATCH_BYTES on each
 * device the library runs on, held until the process ends.  The call makes no
 * device or pinned-host allocation and builds no table: the shared tables
 * must already cover the queries, as after pc_workspace_bytes(xs, n) or any
 * batch of the same queries.  It returns once d_out is complete (it waits for
 * the stream).  Every call on one device shares that device's array and
 * keeps the last call's contents; calls are serialised and each waits for its
 * own work, so calls through this library never overlap, but kernels of
 * another copy of the library in the same process would race on it.
 * Errors: n = 0 is valid and touches nothing; d_xs or d_out null with n > 0
 * -> PC_EINVAL; tables not built or too small for these x, or an x whose
 * sieve counts exceed half the array (x of a few times 10^15 and above)
 * -> PC_ERANGE; more than PC_NOALLOC_SCRATCH_BYTES / 48 queries or a
 * workspace beyond the array -> PC_ENOMEM; these write nothing.  An
 * inconsistency found on the device -> PC_EINTERNAL, with all ones in d_out
 * for the queries of the round where it was found (pi(x) < 2^63 for every
 * x < 2^64, so no count has that value). */
#define PC_NOALLOC_SCRATCH_BYTES (128ull << 20)
pc_status pc_pi_count_batch_noalloc(const uint64_t *d_xs, size_t n, uint64_t *d_out,
                                    void *hip_stream);

/* Serving: an open-loop stream of pi(x) requests replayed in real time, with
 * continuous batching.  Request i (x = xs[i]) arrives arrival_s[i] seconds
 * after the call starts (non-decreasing, finite, >= 0).  Arrived requests wait
 * in order; whenever one of max_inflight slots (a stream and its buffers) is
 * free and the device-memory budget allows, the waiting requests go to the
 * device as one batch round (as pc_pi_count_batch), so later arrivals overlap
 * the rounds already running.  A request whose per-segment counts exceed a
 * round's budget runs alone, windowed, beside the rounds.  pi_out[i] = pi(xs[i])
 * (identical to pc_pi_count), latency_s_out[i] (may be NULL) = completion -
 * arrival on the host clock.  max_inflight = max_round = 1 is the plain
 * per-query server.  Host arrays of n elements; outputs written only on PC_OK. */
typedef struct {
    uint32_t max_inflight; /* batch rounds on the device at once, 1..16; 0 = 3            */
    uint32_t max_round;    /* requests per round; 0 = 4096                                 */
    uint64_t mem_budget;   /* device bytes for the counts of the rounds in flight; 0 = 18 GiB */
    double alpha;          /* y = alpha * icbrt(x) for every request; 0 = tuned             */
    uint32_t flags;        /* PC_FLAG_NO_GRAPH                                              */
    uint32_t pad;
} pc_serve_config;

typedef struct {
    double wall_s;              /* start of the replay to the last completion          */
    uint64_t rounds;            /* batch rounds launched                                */
    uint64_t windowed;          /* requests run alone through the windowed path         */
    uint64_t max_round_size;    /* most requests in one round                           */
    uint64_t max_inflight_seen; /* most rounds on the device at once                    */
    uint64_t device_bytes;      /* peak device bytes held by the library                */
} pc_serve_stats;

pc_status pc_serve(const uint64_t *xs, const double *arrival_s, size_t n,
                   const pc_serve_config *cfg, uint64_t *pi_out, double *latency_s_out,
                   pc_serve_stats *stats);

/* Read-out of the shared device tables that every query uses (the primes and
 * pi(.) of Section 2.1, mu(n) * lpf(n) of Section 2.2), for checking them
 * against an independent computation.  which selects the table; entries
 * lo .. lo + n - 1 are copied to the host array out (n elements):
 *   PC_TABLE_PRIMES  uint32_t: out[i] = p_{lo+i}, the primes 1-based (p_1 = 2);
 *                    lo >= 1, p_{lo+n-1} < 2^32;
 *   PC_TABLE_PI      uint64_t: out[i] = pi(lo + i); lo + n - 1 < 2^32;
 *   PC_TABLE_MULPF   int32_t:  out[i] = mu(v) * lpf(v), v = lo + i: 0 if v = 0
 *                    or v is not squarefree, INT32_MAX at v = 1;
 *                    lo + n - 1 <= 2^31 - 2.
 * The tables are built (or grown) as a query that needs the range would build
 * them.  n = 0 is valid and touches nothing; out null with n > 0, an unknown
 * table or a range outside the table's domain gives PC_EINVAL. */
#define PC_TABLE_PRIMES 1
#define PC_TABLE_PI 2
#define PC_TABLE_MULPF 3
pc_status pc_read_table(int which, uint64_t lo, uint64_t n, void *out);

/* The seeds of a sieve started at m (Section 4, the values phi(m_min, b) that
 * let a block of the sieve run without the blocks before it): out[b - c] =
 * phi(m, b) for c <= b <= b_hi, phi(m, b) = #{1 <= n <= m : no p_i, i <= b,
 * divides n} (Section 3).  Computed on the device from the wheel's phi(m, c)
 * by the recurrence eq. (4.1), each term closed where Section 4's rules close
 * it (a single survivor past pi(sqrt m); Legendre's pi(u) - b + 2 from the pi
 * table) and otherwise expanded by eq. (4.1) again, depth first.  This is
 * what PC_FLAG_SEEDED runs for every window of segments but the first.
 * c: the wheel size, 1 <= c <= pc_wheel_c(), c <= b_hi; m <= 2^48 and
 * b_hi < 2^27 (else PC_ERANGE); out: b_hi - c + 1 host words (null ->
 * PC_EINVAL).  Grows the shared tables as needed (the pi table to m^(2/3)). */
pc_status pc_phi_seed(uint64_t m, uint32_t c, uint32_t b_hi, uint64_t *out);

/* Wheel size c used by the library (c = min(pc_wheel_c(), a)). */
int pc_wheel_c(void);

/* Static text for a status code. */
const char *pc_status_str(pc_status s);

/* Thread-local description of the last error on this thread ("" if none). */
const char *pc_last_error(void);

/* Release every cached device table.  Safe to call at any time between calls. */
void pc_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* PICOUNT_H */

// pc_internal.h -- structures shared between the host planner and the kernel
// launchers of the prime-counting library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pc_device.h"

// One sieve tile: segment `seg` (absolute index), responsible for the
// per-segment columns [col_lo, col_hi).  Column j < nb stands for the sieving
// prime b = c + 1 + j; column nb is the state after every sieving prime is
// crossed (read by the P2 lookups).
struct pc_tile {
    uint32_t seg;
    uint32_t col_lo;
    uint32_t col_hi;
    uint32_t q;             // query (index into the launch's query array)
};

// Shared device tables (read-only during a query).
struct pc_tables {
    const uint32_t *primes; // primes[k] = p_k, 1-based (primes[1] = 2), p_k < 2^32
    const uint64_t *primes_hi; // p_k for k >= k32 (the primes above 2^32): primes_hi[k - k32]
    uint64_t k32;           // index of the first prime above 2^32 (UINT64_MAX: none tabulated)
    const uint64_t *recip;  // recip[k] = floor((2^64-1)/p_k) for k <= n_recip
    const double *rcpd;     // rcpd[k] = 1/p_k correctly rounded, k <= n_recip
    const uint2 *pitab;     // pi table, see pc_pi_lookup
    const int32_t *mulpf;   // mu(n)*lpf(n) for n <= ymax; INT32_MAX at n = 1; 0 if mu = 0
    const uint32_t *pattern; // odd-only pre-sieve bits for p_2..p_c, period pattern_bits (+64 bits)
    const uint32_t *phitab; // phi(r, c) for r < Q_c
    const uint32_t *wres;   // the residues r < Q_c prime to p_1..p_c, ascending (phi(Q_c, c) of them)
    uint32_t pattern_bits;  // prod_{2 <= i <= c} p_i
    uint32_t Qc;            // prod_{1 <= i <= c} p_i
    uint32_t phiQ;          // phi(Q_c, c)
    float rphiQ;            // 1 / phi(Q_c, c)
};

struct pc_sums;

// Per-query scalars.
struct pc_query {
    uint64_t x, y, z;       // x: its low 64 bits when x_hi != 0
    uint64_t x_hi;          // x = x_hi 2^64 + x, x <= 2^72
    double xd;              // x rounded to double
    uint64_t y1, recip_y1;  // y + 1 and its reciprocal
    uint64_t sqrtx;         // isqrt(x)
    uint64_t sqrty;         // isqrt(y): p_b^2 > y  <=>  p_b > sqrty
    uint64_t Qc, recip_Qc;
    uint32_t c, a, bmax, nb, ncol;
    uint32_t kx;            // pi(isqrt(x))
    const uint64_t *Xb;     // Xb[b] = floor(x / p_b) modulo 2^64, 1-based, b <= a
    uint32_t *Xbh;          // its high word (above 2^64; null: every X_b < 2^64)
    uint64_t sieve_end;     // the sieve covers [0, sieve_end): segments * 2S integers
    uint64_t nseg;          // segments (rows of cnt and wgt when the query has one window)
    const ulonglong2 *Ub;   // Ub[b].x <= u of every hard leaf of b <= Ub[b].y, and Ub[b].y is
                            // also >= that bound for every later sieving prime (x > y: none)
    pc_sums *sums;          // device accumulators of this query
    // Sieve counts and leaf weights of the sieving columns j < nb, stored as a
    // staircase: row r (= seg - seg0) holds columns [0, row_off[r+1] -
    // row_off[r]) from row_off[r] on, a bound on the columns that still have
    // a hard leaf at or above the row's first integer (it never grows with r);
    // row_off null: every row holds all nb columns, row r from r nb on.
    const uint64_t *row_off;
    uint32_t *cnt;          // unsieved count before p_b is crossed
    int32_t *wgt;           // sum of -mu(m) over the leaves of the column in the row
    const uint64_t *carry;  // PC_MODE_LEAVES: exclusive carries, same layout
    uint32_t *cntP;         // per row: the count after the last crossing (P2 column)
    int32_t *wP;            // per row: the P2 terms landing in the row
    const uint64_t *carryP; // PC_MODE_LEAVES: exclusive carries of cntP
    // Easy leaves per b (pc_leaf_setup_item), in three kinds:
    //   candidates (p_b^2 <= y): the integers m prime to p_1..p_c, by their
    //     wheel numbers k = e_start[b] .. + e_count[b] - 1 (pc_wheel_m; bit 63
    //     of e_count set), e_off the exclusive prefix of e_count over b and
    //     e_total[0] its total;
    //   singles (p_b^2 > y): primes p_k, k = e_start[b] .. + e_scount[b] - 1;
    //   groups (p_b^2 > y): e_clu[b] = {nk, klo, z, w}, K = klo .. klo + nk
    //     (none when nk = 0).
    // Singles and groups are dealt out in bands of PC_EZ_BAND consecutive b:
    // unit j of band g is the 256 prime indices from e_bk[g] + 256 j on, each
    // taken against every b of the band.  e_bk[g] / e_boff[g] (g < nband):
    // first k and exclusive prefix of the units of the singles; at nband + g
    // the same for the groups; e_total[1] / e_total[2] the units.  Xd[b] =
    // X_b rounded to double.
    uint64_t *e_start;
    uint64_t *e_count;
    uint64_t *e_off;
    uint64_t *e_scount;
    uint4 *e_clu;
    uint32_t *e_bk;
    uint64_t *e_boff;
    double *Xd;
    uint64_t *e_total;
    ulonglong2 *Ub_w;       // writable view of Ub (set-up kernels)
    uint64_t *Xb_w;         // writable view of Xb (set-up kernels)
};

// X_b of a query: its low word, high word and value in fp64 (above 2^64 the
// high word is nonzero for the primes p_b below x / 2^64).
struct pc_xv {
    uint64_t lo;
    uint32_t hi;
    double d;
};

__device__ __forceinline__ pc_xv pc_xb(const pc_query &Q, uint32_t b)
{
    pc_xv v;
    v.lo = Q.Xb[b];
    v.hi = Q.Xbh ? Q.Xbh[b] : 0u;
    v.d = Q.x_hi ? Q.Xd[b] : (double)v.lo;
    return v;
}

// floor(X / p) for a prime p > X's high word (X / p < 2^64), rp = pc_recip(p)
__device__ __forceinline__ uint64_t pc_xv_div(pc_xv X, uint32_t p, uint64_t rp)
{
    return X.hi ? pc_div_wide32(X.hi, X.lo, p, nullptr) : pc_div(X.lo, p, rp);
}

// floor(X / d) for d < 2^46 when the quotient is below 2^64, rd = pc_recip(d)
__device__ __forceinline__ uint64_t pc_xv_div64(pc_xv X, uint64_t d, uint64_t rd)
{
    return X.hi ? pc_div_wide(X.lo, X.d, d) : pc_div(X.lo, d, rd);
}

// floor(X / m) for m < 2^32 when the quotient is below 2^50
__device__ __forceinline__ uint64_t pc_xv_small_q(pc_xv X, uint32_t m)
{
    return X.hi ? pc_div_small_qd(X.lo, X.d, m) : pc_div_small_q(X.lo, m);
}

enum { PC_MODE_TALLY = 0, PC_MODE_COUNT = 1, PC_MODE_LEAVES = 2 };

// b per band of the singles and groups of the easy leaves; bands of a query:
// a / PC_EZ_BAND + 1.
#define PC_EZ_BAND 64
#define PC_EZ_UNIT 256

// per-tile trace record: 0 ticks (100 MHz), 1 hard leaves, 2 candidates read,
// 3 leafy columns, 4 of them with p^3 < segment end, 5.. phase ticks
#define PC_TRACE_W 16

struct pc_sieve_args {
    pc_tables T;
    const pc_query *Qs;     // device array; tile.q indexes it
    const pc_tile *tiles;
    uint32_t ntiles;
    uint32_t pad;
    uint64_t seg0;          // first segment of the window: row = seg - seg0
    uint64_t lo_base;       // segment seg starts at lo_base + (seg - seg_base) * 2S
    uint64_t seg_base;
    pc_s128 *part_hard;     // per tile; null: added to the tile's query sums instead
    pc_s128 *part_p2;       // per tile (null as part_hard)
    int32_t *err;
    uint32_t *trace;        // optional, PC_TRACE_W words per tile (profiling aid)
};

// Launchers (each returns hipSuccess or the first HIP error).
hipError_t pc_launch_base_primes(uint32_t *base, uint32_t *nbase, hipStream_t s);
hipError_t pc_launch_pitab(uint64_t nentries, const uint32_t *base, uint32_t nbase,
                           uint32_t *bits, uint32_t *cnts, uint2 *pitab, uint32_t *primes,
                           uint64_t *primes_hi, uint32_t *scan_tmp, hipStream_t s);
hipError_t pc_launch_recip(const uint32_t *primes, uint64_t *recip, double *rcpd, uint32_t n,
                           hipStream_t s);
hipError_t pc_launch_mulpf(const uint32_t *primes, uint32_t nsmall, uint64_t ymax,
                           int32_t *mulpf, hipStream_t s);
hipError_t pc_launch_count_nonzero(const int32_t *a, uint64_t n, unsigned long long *out,
                                   hipStream_t s);
hipError_t pc_launch_wheel(uint32_t c, const uint32_t *primes, uint32_t *pattern,
                           uint32_t pattern_words, uint32_t *phitab, uint32_t *wres,
                           hipStream_t s);
hipError_t pc_launch_lookup(const uint2 *pitab, const uint64_t *in, uint32_t n, uint64_t *out,
                            hipStream_t s);
hipError_t pc_launch_xb(const pc_tables &T, const pc_query &Q, hipStream_t s);

// Leaves outside the sieve: S1, trivial and easy special leaves.  The set-up
// and easy kernels use the per-query arrays named in pc_query.
hipError_t pc_launch_s1(const pc_tables &T, const pc_query &Q, pc_s128 *part, uint32_t nblocks,
                        hipStream_t s);
hipError_t pc_launch_leaf_setup(const pc_tables &T, const pc_query &Q, pc_s128 *part_trivial,
                                uint32_t nblocks, hipStream_t s);
hipError_t pc_launch_strip(const uint64_t *e_count, uint64_t *e_off, uint64_t n, hipStream_t s);
hipError_t pc_launch_scan_u64(uint64_t *data, uint64_t n, uint64_t *tmp, uint64_t *total,
                              hipStream_t s);
hipError_t pc_launch_easy(const pc_tables &T, const pc_query &Q, pc_s128 *part, uint32_t nblocks,
                          hipStream_t s);
hipError_t pc_launch_easy_bands(const pc_tables &T, const pc_query &Q, hipStream_t s);
hipError_t pc_launch_easy_band(const pc_tables &T, const pc_query &Q, pc_s128 *part,
                               uint32_t nblocks, hipStream_t s);
hipError_t pc_launch_sum128(const pc_s128 *part, uint32_t n, pc_s128 *acc, hipStream_t s);
hipError_t pc_launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);

// Tile planning: hard-leaf items per segment, and column cuts for hot segments.
hipError_t pc_launch_seg_work(const pc_tables &T, const pc_query &Q, uint32_t seg_log2,
                              uint64_t lo_base, uint64_t seg_base, uint64_t seg0, uint32_t nseg,
                              uint64_t *work, hipStream_t s);
hipError_t pc_launch_seg_split(const pc_tables &T, const pc_query &Q, uint32_t seg_log2,
                               uint64_t lo_base, uint64_t seg_base, const uint4 *hot,
                               uint32_t nhot, uint32_t *bounds, hipStream_t s);

// Sieve and carry scan.
hipError_t pc_launch_sieve(const pc_sieve_args &A, uint32_t seg_log2, uint32_t wg, int mode,
                           hipStream_t s);
// The carries of one window: per sieving column an exclusive scan of the
// staircase rows (decoupled look-back over chunks of rows), and the same for
// the P2 column (cntP, one workgroup).  Workgroup tickets run chunk by chunk;
// chunk k has blkoff[k+1] - blkoff[k] blocks of 256 columns (those below the
// chunk's first row length).
struct pc_scan_args {
    const uint32_t *cnt;
    const int32_t *wgt;
    const uint64_t *row_off;  // nrows + 1 (staircase, as pc_query)
    const uint32_t *blkoff;   // nchunk + 1: first ticket of each chunk
    uint64_t *carry_rows;     // PC_MODE_COUNT: exclusive carries, staircase layout
    const uint32_t *cntP;
    const int32_t *wP;
    uint64_t *carryP;         // PC_MODE_COUNT: exclusive carries of cntP
    const uint64_t *carry_in; // per column (nb + 1, the last one P2), from earlier windows
    uint64_t *carry_out;      // per column, for the next window
    uint64_t *status;         // [blkoff[nchunk] * 256] look-back words, zeroed
    uint32_t *ticket;         // zeroed
    pc_s128 *part_hard;       // per ticket
    pc_s128 *part_p2;         // one
    int32_t *err;
    uint64_t nrows;
    uint32_t nb;
    uint32_t rows_per_chunk;  // at most 1024
    uint32_t nchunk;          // ceil(nrows / rows_per_chunk)
    uint32_t nticket;         // blkoff[nchunk]
};
hipError_t pc_launch_scan(const pc_scan_args &A, int mode, hipStream_t s);

// The seeds of a window that starts at m (Section 4): out[j] = phi(m, c + j)
// for 0 <= j <= nb, from phi(m, c) by eq. (4.1), each term closed (one left,
// Legendre from the pi table) or expanded depth first.  T's wheel is of size
// c; T's primes and reciprocals cover p_{c+nb}; the pi table covers
// m^(2/3) (pi_limit, else err |= 16); m <= 2^48.  nrec >= the columns j with
// p_{c+j}^3 <= m (one workgroup each); term: nb + 1 words of scratch.
hipError_t pc_launch_seed(const pc_tables &T, uint32_t c, uint64_t m, uint32_t nb,
                          uint32_t nrec, uint64_t pi_limit, int64_t *term, uint64_t *out,
                          int32_t *err, hipStream_t s);

// Final combination of the partial sums into pi(x) and its parts.
struct pc_sums {
    pc_s128 s1, s2t, s2e, hard_local, hard_dot, p2_local, p2_dot;
    unsigned long long n_s1, n_easy, n_hard, crossings, n_trivial;
    unsigned long long n_easy_terms; // singles and group terms of the easy leaves
};
struct pc_final {
    pc_s128 s1, s2t, s2e, s2h, p2, phi;
    uint64_t pi, pi_hi;     // pi(x) = pi_hi 2^64 + pi
    uint64_t ok;            // 1: pi in [0, 2^64); 2: pi in [2^64, 2^128); 0: negative
    uint64_t pad;
};
// Batches: the queries' set-up (X_b, S1, per-b leaf set-up, easy offsets),
// their easy leaves, and their carries and combination, each over all queries
// of the batch.  bq / bf: the query of each block, the first block of each
// query (bf[nq] = blocks).
hipError_t pc_launch_batch_setup(const pc_tables &T, const pc_query *Qs, const uint32_t *bq_xb,
                                 const uint32_t *bf_xb, uint32_t nb_xb, const uint32_t *bq_s1,
                                 const uint32_t *bf_s1, uint32_t nb_s1, uint32_t nq,
                                 hipStream_t s);
hipError_t pc_launch_batch_easy(const pc_tables &T, const pc_query *Qs, const uint32_t *bq,
                                const uint32_t *bf, uint32_t nblocks, hipStream_t s);
hipError_t pc_launch_batch_finish(const pc_query *Qs, const uint32_t *bq, const uint32_t *bf,
                                  uint32_t nblocks, uint32_t nq, pc_final *out, hipStream_t s);
// The caller-memory batch path: a round's results, and results known on the
// host ((position, value) pairs), written into the caller's output array.
hipError_t pc_launch_batch_out(const pc_final *fin, const uint64_t *pos, uint32_t nq,
                               const int32_t *err, uint64_t *out, hipStream_t s);
hipError_t pc_launch_scatter_u64(const ulonglong2 *kv, uint64_t n, uint64_t *out, hipStream_t s);

hipError_t pc_launch_combine(const pc_sums *sums, const pc_query &Q, uint64_t kp2,
                             pc_final *out, hipStream_t s);

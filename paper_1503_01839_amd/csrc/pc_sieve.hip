// pc_sieve.hip -- the hot path: a segmented sieve of [1, z], z = floor(x/y),
// that reads phi(u, b-1) for every hard special leaf and pi(x/p) for every P2
// term (Sections 2.3 and 3 of the paper; the counters, blocks and per-prime
// running values phi(m_min, b) that Section 3 and Section 4 describe).
//
// Layout.  A segment holds S odd integers as an LDS bitmap: bit i <-> the
// integer seg*2S + 2i + 1 (p_1 = 2 is implicit).  Column j < nb stands for the
// sieving prime b = c + 1 + j (p_{c+1} .. p_bmax, bmax = pi(isqrt z)); column
// nb is the state after every sieving prime is crossed.  For every
// (segment, column) the kernel records
//   cnt = the number of integers of the segment still unsieved just before
//         p_b is crossed (column nb: after the last crossing), and
//   w   = the sum of -mu(m) over the leaves of that column whose u lands in
//         the segment (column nb: the number of P2 terms landing there),
// and it sums -mu(m) * (unsieved integers of the segment that are <= u).
// phi(u, b-1) is that in-segment count plus carry = sum of cnt over the
// earlier segments in the same column, so the carry part of the hard-leaf
// sum is sum w * carry, formed by the look-back scan below (one sieve pass
// instead of a count pass and a leaf pass; PC_MODE_COUNT / PC_MODE_LEAVES run
// the two-pass form for cross-checking).
//
// Crossing p_b clears every odd multiple k p_b, k >= 1, including p_b itself:
// phi(u, b) counts integers coprime to p_1..p_b, so p_b must go (unlike a
// prime sieve).  Per column the workgroup first answers the leaves, then
// crosses.  Columns are processed in order; for primes with p^3 >= hi (every
// unsieved integer below the segment end then has at most two prime factors
// >= p) a run of columns without leaves is crossed in one step, one lane per
// prime: an integer n = p k unsieved at the start of the run is first removed
// by p exactly when k = 1 or k >= p, which gives the per-column counts
// without ordering the lanes.
#include "pc_block.h"
#include "pc_internal.h"

#define PC_CAND 0x80000000u

template <int LOG2_S, int T, int CH, int MODE, bool BATCH>
__global__ __launch_bounds__(T) void k_sieve(pc_sieve_args A)
{
    static_assert(T >= CH, "one lane per column of a chunk");
    static_assert(CH % 64 == 0 && T % 64 == 0, "wavefront multiples");
    constexpr uint32_t S = 1u << LOG2_S;      // odd integers per segment
    constexpr uint32_t NW = S / 32;           // 32-bit words
    constexpr uint32_t BL = 9;                // 512-bit counting blocks
    constexpr uint32_t NBLK = S >> BL;
    constexpr uint32_t NWV = T / 64;
    constexpr uint32_t PER = NBLK >= T ? NBLK / T : 1;

    __shared__ uint64_t bm64[NW / 2];
    __shared__ uint32_t blkcnt[NBLK];
    __shared__ uint32_t blkpre[NBLK + 1];
    __shared__ uint32_t c_p[CH];   // p_b
    __shared__ uint32_t c_i0[CH];  // bit of the first multiple in the segment, S if none
    __shared__ uint32_t c_ls[CH];  // first leaf item (m, or index of the prime m)
    __shared__ uint32_t c_lc[CH];  // leaf items; PC_CAND: items are candidate m
    __shared__ uint32_t c_new[CH]; // integers first removed by p_b in this segment
    __shared__ int32_t c_w[CH];    // sum of -mu(m) over the leaves of the column
    __shared__ uint64_t c_leafy[CH / 64];
    __shared__ uint32_t s_first_large;
    __shared__ uint32_t scr32[NWV];
    __shared__ pc_s128 scr128[NWV];
    uint32_t *bm = (uint32_t *)bm64;

    const pc_tile tile = A.tiles[blockIdx.x];
    const uint32_t tid = threadIdx.x;
    const uint64_t seg = tile.seg;
    const uint64_t lo = seg << (LOG2_S + 1);
    const uint64_t hi = lo + (2ull << LOG2_S);
    const uint64_t row = seg - A.seg0;
    const pc_query &Q = A.Q;
    const pc_tables &TB = A.T;
    const uint64_t rhi = pc_recip(hi);
    const uint64_t rlo = lo ? pc_recip(lo) : 0;
    const uint32_t ncol = Q.ncol;

    // --- pre-sieved state: the wheel pattern (p_2..p_c already crossed) ---
    {
        const uint32_t P = TB.pattern_bits;
        const uint32_t g0 = (uint32_t)((seg << LOG2_S) % P);
        for (uint32_t w = tid; w < NW; w += T) {
            uint32_t off = (g0 + 32u * w) % P;
            uint32_t wi = off >> 5, sh = off & 31;
            uint32_t v = TB.pattern[wi] >> sh;
            if (sh)
                v |= TB.pattern[wi + 1] << (32 - sh);
            bm[w] = v;
        }
    }
    __syncthreads();
    uint32_t total;
    {
        uint32_t mine = 0;
        for (uint32_t k = tid; k < NBLK; k += T) {
            uint32_t s = 0;
#pragma unroll
            for (int j = 0; j < 8; j++)
                s += (uint32_t)__builtin_popcountll(bm64[k * 8 + j]);
            blkcnt[k] = s;
            mine += s;
        }
        total = pc_block_sum<T>(mine, scr32);
    }

    // exclusive prefix of the block counts -> blkpre (blkpre[NBLK] = total)
    auto rebuild = [&]() {
        uint32_t s = 0;
        const uint32_t b0 = tid * PER;
        if (b0 < NBLK)
            for (uint32_t k = 0; k < PER; k++)
                s += blkcnt[b0 + k];
        uint32_t tot;
        uint32_t ex = pc_block_excl_scan<T>(s, scr32, &tot);
        if (b0 < NBLK)
            for (uint32_t k = 0; k < PER; k++) {
                blkpre[b0 + k] = ex;
                ex += blkcnt[b0 + k];
            }
        if (tid == 0)
            blkpre[NBLK] = tot;
        __syncthreads();
    };
    // unsieved integers among bits [0, q), q <= S
    auto count_below = [&](uint32_t q) -> uint32_t {
        const uint32_t blk = q >> BL;
        uint32_t s = blkpre[blk];
        const uint32_t w64 = q >> 6;
        for (uint32_t i = blk << (BL - 6); i < w64; i++)
            s += (uint32_t)__builtin_popcountll(bm64[i]);
        const uint32_t r = q & 63;
        if (r)
            s += (uint32_t)__builtin_popcountll(bm64[w64] & ((1ull << r) - 1));
        return s;
    };

    int64_t acc_local = 0; // sum of -mu(m) * in-segment count (hard leaves)
    int64_t acc_p2 = 0;    // sum of in-segment counts (P2 terms)
    pc_s128 acc_carry = 0; // PC_MODE_LEAVES: carry * w, kept by thread 0

    const uint32_t col_lo = tile.col_lo, col_hi = tile.col_hi;
    const uint32_t ncross = min(col_hi, Q.nb);
    for (uint32_t cb = 0; cb < ncross; cb += CH) {
        const uint32_t jend = min((uint32_t)CH, ncross - cb);
        if (tid == 0)
            s_first_large = jend;
        __syncthreads();
        // --- phase A: one lane per column: first multiple, leaf range ---
        bool leafy = false;
        if (tid < jend) {
            const uint32_t j = tid, col = cb + j, b = Q.c + 1 + col;
            const uint64_t p = TB.primes[b];
            const uint64_t rp = TB.recip[b];
            c_p[j] = (uint32_t)p;
            uint64_t first;
            if (lo <= p) {
                first = p;
            } else {
                uint64_t m = pc_div(lo, p, rp) * p;
                if (m < lo)
                    m += p;
                if ((m & 1) == 0)
                    m += p;
                first = m;
            }
            c_i0[j] = first < hi ? (uint32_t)((first - lo - 1) >> 1) : S;
            if ((pc_u128)p * p * p >= hi)
                atomicMin(&s_first_large, j);
            uint32_t ls = 0, lc = 0;
            if (MODE != PC_MODE_COUNT && col >= col_lo && col < col_hi) {
                const uint64_t X = Q.Xb[b];
                // u = floor(X/m) lies in [lo, hi)  <=>  X/hi < m <= X/lo
                const uint64_t mA = pc_div(X, hi, rhi) + 1;
                const uint64_t mB = lo ? pc_div(X, lo, rlo) : X;
                // special leaf: y/p_b < m <= y, lpf(m) > p_b; hard: m <= max(x/p^3, x/(p(y+1)))
                uint64_t m1 = pc_div(Q.y, p, rp) + 1;
                if (m1 < mA)
                    m1 = mA;
                if (m1 < p + 1)
                    m1 = p + 1;
                const uint64_t h1 = pc_div(pc_div(X, p, rp), p, rp);
                const uint64_t h2 = pc_div(X, Q.y1, Q.recip_y1);
                uint64_t m2 = h1 > h2 ? h1 : h2;
                if (m2 > Q.y)
                    m2 = Q.y;
                if (m2 > mB)
                    m2 = mB;
                if (m1 <= m2) {
                    if (p > Q.sqrty) { // p^2 > y: every such m is a prime
                        const uint32_t k1 = pc_pi_lookup(TB.pitab, m1 - 1) + 1;
                        const uint32_t k2 = pc_pi_lookup(TB.pitab, m2);
                        if (k1 <= k2) {
                            ls = k1;
                            lc = k2 - k1 + 1;
                        }
                    } else {
                        ls = (uint32_t)m1;
                        lc = (uint32_t)(m2 - m1 + 1) | PC_CAND;
                    }
                }
            }
            c_ls[j] = ls;
            c_lc[j] = lc;
            c_new[j] = 0;
            c_w[j] = 0;
            leafy = lc != 0;
        }
        {
            const uint64_t bal = __ballot(leafy);
            if ((tid & 63) == 0 && tid < CH)
                c_leafy[tid >> 6] = bal;
        }
        __syncthreads();

        // --- phase B: columns in order ---
        const uint32_t first_large = BATCH ? s_first_large : jend;
        uint32_t j = 0;
        while (j < jend) {
            const bool lf = (c_leafy[j >> 6] >> (j & 63)) & 1;
            if (j < first_large || lf) {
                if (lf) {
                    rebuild();
                    const uint32_t b = Q.c + 1 + cb + j;
                    const uint32_t lc = c_lc[j], ls = c_ls[j], p = c_p[j];
                    const bool cand = (lc & PC_CAND) != 0;
                    const uint32_t n = lc & ~PC_CAND;
                    const uint64_t X = Q.Xb[b];
                    int32_t wsum = 0;
                    int64_t lsum = 0;
                    for (uint32_t t2 = tid; t2 < n; t2 += T) {
                        uint64_t u;
                        int32_t w;
                        if (cand) {
                            const uint32_t m = ls + t2;
                            const int32_t v = TB.mulpf[m];
                            const uint32_t av = v < 0 ? (uint32_t)(-v) : (uint32_t)v;
                            if (av <= p) // mu(m) = 0 or lpf(m) <= p_b
                                continue;
                            w = v > 0 ? -1 : 1;
                            u = pc_div_small_q(X, m);
                        } else {
                            const uint32_t k = ls + t2;
                            u = pc_div(X, TB.primes[k], TB.recip[k]);
                            w = 1;
                        }
                        if (u < lo || u >= hi) { // cannot happen if the m range is right
                            atomicOr(A.err, 2);
                            continue;
                        }
                        const uint32_t q = (uint32_t)((u - lo + 1) >> 1);
                        lsum += (int64_t)w * (int64_t)count_below(q);
                        wsum += w;
                    }
                    acc_local += lsum;
                    wsum = pc_wave_sum(wsum);
                    if ((tid & 63) == 0 && wsum != 0)
                        atomicAdd(&c_w[j], wsum);
                    __syncthreads();
                    if (MODE == PC_MODE_LEAVES && tid == 0)
                        acc_carry += (pc_s128)c_w[j] *
                                     (pc_s128)A.carry[row * ncol + cb + j];
                }
                const uint32_t i0 = c_i0[j];
                if (i0 < S) {
                    const uint32_t p = c_p[j];
                    const uint32_t n = (S - 1 - i0) / p + 1;
                    uint32_t mine = 0;
                    for (uint32_t t2 = tid; t2 < n; t2 += T) {
                        const uint32_t bit = i0 + t2 * p;
                        const uint32_t mask = 1u << (bit & 31);
                        const uint32_t old = atomicAnd(&bm[bit >> 5], ~mask);
                        if (old & mask) {
                            mine++;
                            atomicSub(&blkcnt[bit >> BL], 1u);
                        }
                    }
                    mine = pc_wave_sum(mine);
                    if ((tid & 63) == 0 && mine)
                        atomicAdd(&c_new[j], mine);
                    __syncthreads();
                }
                j++;
            } else {
                // run of leafless columns [j, jb), all with p^3 >= hi
                uint32_t jb = jend;
                {
                    uint32_t wv = j >> 6;
                    uint64_t msk = c_leafy[wv] & (~0ull << (j & 63));
                    while (!msk && ++wv < (jend + 63) / 64)
                        msk = c_leafy[wv];
                    if (msk)
                        jb = min(jend, wv * 64 + (uint32_t)__builtin_ctzll(msk));
                }
                const uint32_t jj = j + tid;
                const bool mine_col = jj < jb;
                uint32_t i0 = S, p = 0;
                if (mine_col) {
                    i0 = c_i0[jj];
                    p = c_p[jj];
                }
                // read: credit n = p k to p when k = 1 or k >= p
                if (mine_col) {
                    uint32_t credit = 0;
                    const uint64_t p2 = (uint64_t)p * p;
                    for (uint32_t bit = i0; bit < S; bit += p)
                        if ((bm[bit >> 5] >> (bit & 31)) & 1) {
                            const uint64_t nn = lo + 2ull * bit + 1;
                            credit += (nn == p || nn >= p2) ? 1u : 0u;
                        }
                    c_new[jj] = credit;
                }
                __syncthreads();
                // clear
                if (mine_col)
                    for (uint32_t bit = i0; bit < S; bit += p) {
                        const uint32_t mask = 1u << (bit & 31);
                        const uint32_t old = atomicAnd(&bm[bit >> 5], ~mask);
                        if (old & mask)
                            atomicSub(&blkcnt[bit >> BL], 1u);
                    }
                __syncthreads();
                j = jb;
            }
        }
        // --- chunk results: cnt before each crossing, and w ---
        {
            const uint32_t v = tid < jend ? c_new[tid] : 0;
            uint32_t tot;
            const uint32_t ex = pc_block_excl_scan<T>(v, scr32, &tot);
            if (tid < jend) {
                const uint32_t col = cb + tid;
                if (col >= col_lo && col < col_hi) {
                    const uint64_t idx = row * ncol + col;
                    if (MODE != PC_MODE_LEAVES)
                        A.cnt[idx] = total - ex;
                    if (MODE == PC_MODE_TALLY)
                        A.wgt[idx] = c_w[tid];
                }
            }
            total -= tot;
        }
    }

    // --- final column: P2 lookups pi(x/p) = phi(x/p, bmax) + bmax - 1 ---
    pc_s128 extra_p2 = 0; // PC_MODE_LEAVES: carry * (lookups), kept by thread 0
    if (col_hi == ncol) {
        rebuild();
        uint32_t k1 = 1, k2 = 0;
        {
            const uint64_t tA = pc_div(Q.x, hi, rhi);              // x/p < hi  <=> p > x/hi
            const uint64_t tB = lo ? pc_div(Q.x, lo, rlo) : ~0ull; // x/p >= lo <=> p <= x/lo
            const uint64_t pl = tA > Q.y ? tA : Q.y;
            const uint64_t ph = tB < Q.sqrtx ? tB : Q.sqrtx;
            if (pl < ph) {
                k1 = pc_pi_lookup(TB.pitab, pl) + 1;
                k2 = pc_pi_lookup(TB.pitab, ph);
            }
        }
        if (MODE != PC_MODE_COUNT)
            for (uint32_t k = k1 + tid; k <= k2; k += T) {
                const uint64_t v = pc_div_small_q(Q.x, TB.primes[k]);
                if (v < lo || v >= hi) {
                    atomicOr(A.err, 4);
                    continue;
                }
                const uint32_t q = (uint32_t)((v - lo + 1) >> 1);
                acc_p2 += count_below(q);
            }
        if (tid == 0) {
            const uint64_t idx = row * ncol + Q.nb;
            const uint32_t np = k2 >= k1 ? k2 - k1 + 1 : 0;
            if (MODE != PC_MODE_LEAVES)
                A.cnt[idx] = total;
            if (MODE == PC_MODE_TALLY)
                A.wgt[idx] = (int32_t)np;
            if (MODE == PC_MODE_LEAVES)
                extra_p2 = (pc_s128)np * (pc_s128)A.carry[idx];
        }
    }
    if (MODE != PC_MODE_COUNT) {
        const pc_s128 h = pc_block_sum128<T>((pc_s128)acc_local + acc_carry, scr128);
        const pc_s128 q = pc_block_sum128<T>((pc_s128)acc_p2 + extra_p2, scr128);
        if (tid == 0) {
            A.part_hard[blockIdx.x] = h;
            A.part_p2[blockIdx.x] = q;
        }
    }
}

// ---------------------------------------------------------------------------
// Look-back scan over the segments of a window, independently per column:
// carry[s][col] = carry_in[col] + sum_{s' < s} cnt[s'][col].  Workgroups take
// tickets in order; a workgroup owns rows_per_chunk rows of 256 columns,
// publishes its column sums, and looks back through earlier chunks until one
// has published an inclusive prefix (decoupled look-back).  PC_MODE_TALLY
// forms sum w * carry; PC_MODE_COUNT writes the carries out for the leaf pass.
// ---------------------------------------------------------------------------
#define SCAN_T 256
#define LB_A (1ull << 62)
#define LB_P (2ull << 62)
#define LB_V ((1ull << 62) - 1)

template <int MODE> __global__ __launch_bounds__(SCAN_T) void k_scan(pc_scan_args A)
{
    __shared__ uint32_t s_ticket;
    __shared__ pc_s128 scr[SCAN_T / 64];
    if (threadIdx.x == 0)
        s_ticket = atomicAdd(A.ticket, 1u);
    __syncthreads();
    const uint32_t tk = s_ticket;
    const uint32_t rc = tk / A.ncb, cb = tk % A.ncb;
    const uint32_t col = cb * SCAN_T + threadIdx.x;
    const bool act = col < A.ncol;
    const uint64_t r0 = (uint64_t)rc * A.rows_per_chunk;
    const uint64_t r1 = min(r0 + A.rows_per_chunk, A.nrows);
    const uint64_t ncol = A.ncol;
    uint64_t agg = 0, pre = 0;
    if (act) {
        for (uint64_t r = r0; r < r1; r++)
            agg += A.cnt[r * ncol + col];
        uint64_t *st = A.status + (uint64_t)rc * ncol + col;
        if (rc == 0) {
            __hip_atomic_store(st, LB_P | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(st, LB_A | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t jc = (int64_t)rc - 1;
            uint32_t spins = 0;
            while (jc >= 0) {
                const uint64_t v = __hip_atomic_load(A.status + (uint64_t)jc * ncol + col,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t f = v >> 62;
                if (f == 0) {
                    if (++spins > (1u << 26)) { // never expected: earlier tickets always run
                        atomicOr(A.err, 1);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                pre += v & LB_V;
                if (f == 2)
                    break;
                jc--;
            }
            __hip_atomic_store(st, LB_P | ((pre + agg) & LB_V), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    pc_s128 dh = 0, dp = 0;
    if (act) {
        uint64_t carry = A.carry_in[col] + pre;
        for (uint64_t r = r0; r < r1; r++) {
            const uint64_t idx = r * ncol + col;
            if (MODE == PC_MODE_TALLY) {
                const int32_t w = A.wgt[idx];
                if (w) {
                    if (col == A.nb)
                        dp += (pc_s128)w * (pc_s128)carry;
                    else
                        dh += (pc_s128)w * (pc_s128)carry;
                }
            } else {
                A.carry_rows[idx] = carry;
            }
            carry += A.cnt[idx];
        }
        if (rc == A.nchunk - 1)
            A.carry_out[col] = carry;
    }
    if (MODE == PC_MODE_TALLY) {
        dh = pc_block_sum128<SCAN_T>(dh, scr);
        dp = pc_block_sum128<SCAN_T>(dp, scr);
        if (threadIdx.x == 0) {
            A.part_hard[tk] = dh;
            A.part_p2[tk] = dp;
        }
    }
}

hipError_t pc_launch_scan(const pc_scan_args &A, int mode, hipStream_t s)
{
    const uint32_t nwg = A.nchunk * A.ncb;
    if (mode == PC_MODE_TALLY)
        k_scan<PC_MODE_TALLY><<<nwg, SCAN_T, 0, s>>>(A);
    else
        k_scan<PC_MODE_COUNT><<<nwg, SCAN_T, 0, s>>>(A);
    return hipGetLastError();
}

template <int LOG2_S, int T, int CH>
static hipError_t launch_modes(const pc_sieve_args &A, int mode, bool batch, hipStream_t s)
{
    const uint32_t g = A.ntiles;
    if (batch) {
        if (mode == PC_MODE_TALLY)
            k_sieve<LOG2_S, T, CH, PC_MODE_TALLY, true><<<g, T, 0, s>>>(A);
        else if (mode == PC_MODE_COUNT)
            k_sieve<LOG2_S, T, CH, PC_MODE_COUNT, true><<<g, T, 0, s>>>(A);
        else
            k_sieve<LOG2_S, T, CH, PC_MODE_LEAVES, true><<<g, T, 0, s>>>(A);
    } else {
        if (mode == PC_MODE_TALLY)
            k_sieve<LOG2_S, T, CH, PC_MODE_TALLY, false><<<g, T, 0, s>>>(A);
        else if (mode == PC_MODE_COUNT)
            k_sieve<LOG2_S, T, CH, PC_MODE_COUNT, false><<<g, T, 0, s>>>(A);
        else
            k_sieve<LOG2_S, T, CH, PC_MODE_LEAVES, false><<<g, T, 0, s>>>(A);
    }
    return hipGetLastError();
}

hipError_t pc_launch_sieve(const pc_sieve_args &A, uint32_t seg_log2, uint32_t wg, int mode,
                           hipStream_t s)
{
    const bool batch = (mode & 0x100) == 0;
    mode &= 0xFF;
    if (A.ntiles == 0)
        return hipSuccess;
    if (seg_log2 == 18 && wg == 1024)
        return launch_modes<18, 1024, 1024>(A, mode, batch, s);
    if (seg_log2 == 18 && wg == 512)
        return launch_modes<18, 512, 512>(A, mode, batch, s);
    if (seg_log2 == 19 && wg == 1024)
        return launch_modes<19, 1024, 1024>(A, mode, batch, s);
    if (seg_log2 == 19 && wg == 512)
        return launch_modes<19, 512, 512>(A, mode, batch, s);
    if (seg_log2 == 20 && wg == 1024)
        return launch_modes<20, 1024, 256>(A, mode, batch, s);
    if (seg_log2 == 20 && wg == 512)
        return launch_modes<20, 512, 256>(A, mode, batch, s);
    return hipErrorInvalidValue;
}

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

// The hard leaves (b, m) whose u = floor(X_b/m) lies in [lo, hi): special
// (y/p_b < m <= y, lpf(m) > p_b) and hard (m <= max(x/p^3, x/(p(y+1)))).
// For p_b^2 > y every such m is prime and the range is returned as prime
// indices [ls, ls + lc); otherwise as candidate m values, lc | PC_CAND.
__device__ __forceinline__ void pc_leaf_range(const pc_tables &TB, const pc_query &Q, uint32_t b,
                                              uint64_t p, uint64_t rp, uint64_t lo, uint64_t hi,
                                              uint64_t rhi, uint64_t rlo, uint32_t *ls,
                                              uint32_t *lc)
{
    const uint64_t X = Q.Xb[b];
    const uint64_t mA = pc_div(X, hi, rhi) + 1;            // u < hi   <=> m > X/hi
    const uint64_t mB = lo ? pc_div(X, lo, rlo) : X;        // u >= lo  <=> m <= X/lo
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
    *ls = 0;
    *lc = 0;
    if (m1 <= m2) {
        if (p > Q.sqrty) {
            const uint32_t k1 = pc_pi_lookup(TB.pitab, m1 - 1) + 1;
            const uint32_t k2 = pc_pi_lookup(TB.pitab, m2);
            if (k1 <= k2) {
                *ls = k1;
                *lc = k2 - k1 + 1;
            }
        } else {
            *ls = (uint32_t)m1;
            *lc = (uint32_t)(m2 - m1 + 1) | PC_CAND;
        }
    }
}

template <int LOG2_S, int T, int CH, int MODE, bool BATCH>
__global__ __launch_bounds__(T) void k_sieve(pc_sieve_args A)
{
    static_assert(CH == T, "one lane per column of a chunk");
    static_assert(T % 64 == 0, "wavefront multiples");
    constexpr uint32_t S = 1u << LOG2_S;  // odd integers (bits) per segment
    constexpr uint32_t NW = S / 32;       // 32-bit words
    constexpr uint32_t NWP = NW + NW / 16; // padded: one spare word after every 16
    constexpr uint32_t BL = 9;            // 512-bit counting blocks (16 words)
    constexpr uint32_t NBLK = S >> BL;
    constexpr uint32_t NWV = T / 64;
    constexpr uint32_t BPT = NBLK / T;    // blocks a thread owns while crossing small primes
    static_assert(NBLK % T == 0 && BPT >= 1, "every thread owns whole counting blocks");
    constexpr uint32_t OWN = BPT << BL;   // bits owned per thread
    constexpr uint32_t LIGHT = 128;       // leaf items a single wavefront answers per column
    constexpr uint32_t GAP = 4;           // leafless columns that end a single-wavefront run

    // Word w of the segment lives at bm[w + w/16]: the 16 words of a counting
    // block are contiguous and consecutive blocks start 17 words apart, so the
    // threads of a wavefront walking their own blocks hit distinct banks.
    __shared__ uint32_t bm[NWP + 16];  // 16 spare words: a query at q = S reads past the end
    __shared__ uint32_t pre[NBLK + 1];   // prefix of the block counts (pre[NBLK] = total)
    __shared__ uint32_t fen[NBLK + 1];   // Fenwick tree over the blocks, 1-based
    __shared__ uint32_t c_p[CH];         // p_b
    __shared__ uint32_t c_i0[CH];        // bit of the first multiple in the segment, S if none
    __shared__ uint32_t c_ls[CH];        // first leaf item (m, or index of the prime m)
    __shared__ uint32_t c_lc[CH];        // leaf items; PC_CAND: items are candidate m
    __shared__ uint32_t c_new[CH];       // integers first removed by p_b in this segment
    __shared__ int32_t c_w[CH];          // sum of -mu(m) over the leaves of the column
    __shared__ uint64_t c_leafy[CH / 64];
    __shared__ uint64_t c_heavy[CH / 64];
    __shared__ uint32_t s_first_large;
    __shared__ uint32_t scr32[NWV];
    __shared__ pc_s128 scr128[NWV];

    const uint64_t t_start = A.trace ? __builtin_amdgcn_s_memrealtime() : 0;
    uint32_t n_cand = 0, n_leafy = 0;
    const pc_tile tile = A.tiles[blockIdx.x];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    if (tile.col_lo >= tile.col_hi) { // a split that owns no column
        if (MODE != PC_MODE_COUNT && tid == 0) {
            A.part_hard[blockIdx.x] = 0;
            A.part_p2[blockIdx.x] = 0;
        }
        return;
    }
    const uint64_t seg = tile.seg;
    const uint64_t lo = A.lo_base + ((seg - A.seg_base) << (LOG2_S + 1));
    const uint64_t hi = lo + (2ull << LOG2_S);
    const uint64_t row = seg - A.seg0;
    const pc_query &Q = A.Q;
    const pc_tables &TB = A.T;
    const uint64_t rhi = pc_recip(hi);
    const uint64_t rlo = lo ? pc_recip(lo) : 0;
    const uint32_t ncol = Q.ncol;
#define BW(w) bm[(w) + ((w) >> 4)]

    // --- pre-sieved state: the wheel pattern (p_2..p_c already crossed) ---
    {
        const uint32_t P = TB.pattern_bits;
        const uint32_t g0 = (uint32_t)((lo >> 1) % P);
        for (uint32_t w = tid; w < NW; w += T) {
            uint32_t off = (g0 + 32u * w) % P;
            uint32_t wi = off >> 5, sh = off & 31;
            uint32_t v = TB.pattern[wi] >> sh;
            if (sh)
                v |= TB.pattern[wi + 1] << (32 - sh);
            BW(w) = v;
        }
    }
    __syncthreads();

    // pre[] = exclusive prefix of the unsieved counts of the blocks, each thread
    // counting the blocks it owns; returns the segment total.
    auto build_pre = [&]() -> uint32_t {
        uint32_t cnt[BPT], s = 0;
#pragma unroll
        for (uint32_t k = 0; k < BPT; k++) {
            const uint32_t base = (tid * BPT + k) * 17;
            uint32_t c = 0;
#pragma unroll
            for (uint32_t j = 0; j < 16; j++)
                c += (uint32_t)__builtin_popcount(bm[base + j]);
            cnt[k] = c;
            s += c;
        }
        uint32_t tot;
        uint32_t ex = pc_block_excl_scan<T>(s, scr32, &tot);
#pragma unroll
        for (uint32_t k = 0; k < BPT; k++) {
            pre[tid * BPT + k] = ex;
            ex += cnt[k];
        }
        if (tid == 0)
            pre[NBLK] = tot;
        __syncthreads();
        return tot;
    };
    // Fenwick tree from pre[]: fen[i] covers blocks [i - lowbit(i), i) (0-based)
    auto build_fen = [&]() {
        for (uint32_t i = tid + 1; i <= NBLK; i += T)
            fen[i] = pre[i] - pre[i - (i & (0u - i))];
        __syncthreads();
    };
    auto fen_dec = [&](uint32_t blk) {
        for (uint32_t i = blk + 1; i <= NBLK; i += i & (0u - i))
            __hip_atomic_fetch_sub(&fen[i], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // unsieved integers among the bits of q's block below q: the block's 16
    // words are read unconditionally and masked, so the reads issue together
    auto in_block = [&](uint32_t q) -> uint32_t {
        const uint32_t base = (q >> BL) * 17;
        const uint32_t nw = (q >> 5) & 15, r = q & 31;
        const uint32_t part = (1u << r) - 1;
        uint32_t s = 0;
#pragma unroll
        for (uint32_t k = 0; k < 16; k++) {
            const uint32_t m = k < nw ? ~0u : (k == nw ? part : 0u);
            s += (uint32_t)__builtin_popcount(bm[base + k] & m);
        }
        return s;
    };
    // unsieved integers among bits [0, q), q <= S
    auto count_pre = [&](uint32_t q) -> uint32_t { return pre[q >> BL] + in_block(q); };
    // Fenwick prefix over blocks [0, q/512): the node indices depend only on q,
    // so the (at most log2(NBLK)+1) reads are unrolled and issue together
    auto count_fen = [&](uint32_t q) -> uint32_t {
        uint32_t i = q >> BL, s = 0;
#pragma unroll
        for (uint32_t l = 0; l <= LOG2_S - BL; l++) {
            const uint32_t v = fen[i];
            s += i ? v : 0u;
            i &= i - 1;
        }
        return s + in_block(q);
    };

    uint32_t total = build_pre();
    bool fen_ok = false;               // uniform: the Fenwick tree mirrors the bitmap
    unsigned long long nleaf = 0;      // hard leaves answered by this thread
    int64_t acc_local = 0;             // sum of -mu(m) * in-segment count (hard leaves)
    int64_t acc_p2 = 0;                // sum of in-segment counts (P2 terms)
    pc_s128 acc_carry = 0;             // PC_MODE_LEAVES: carry * w, kept by thread 0

    // The leaves of column j (chunk base cb): items t0, t0 + stride, ... of the
    // column; returns this thread's sum of -mu(m).
    auto leaves = [&](uint32_t cb, uint32_t j, bool use_fen, uint32_t t0, uint32_t stride) -> int32_t {
        constexpr uint32_t U = 4; // items in flight per lane
        const uint32_t b = Q.c + 1 + cb + j;
        const uint32_t lc = c_lc[j], ls = c_ls[j], p = c_p[j];
        const bool cand = (lc & PC_CAND) != 0;
        const uint32_t n = lc & ~PC_CAND;
        const uint64_t X = Q.Xb[b];
        int32_t wsum = 0;
        int64_t lsum = 0;
        for (uint32_t t2 = t0; t2 < n; t2 += U * stride) {
            uint32_t mm[U];
            int32_t ww[U];
#pragma unroll
            for (uint32_t k = 0; k < U; k++) { // issue the loads of U items together
                const uint32_t it = t2 + k * stride;
                mm[k] = 0;
                ww[k] = 0;
                if (it < n) {
                    if (cand) {
                        const int32_t v = TB.mulpf[ls + it];
                        const uint32_t av = v < 0 ? (uint32_t)(-v) : (uint32_t)v;
                        if (av > p) { // squarefree with lpf(m) > p_b
                            mm[k] = ls + it;
                            ww[k] = v > 0 ? -1 : 1;
                        }
                    } else {
                        mm[k] = TB.primes[ls + it];
                        ww[k] = 1;
                    }
                }
            }
            if (cand)
#pragma unroll
                for (uint32_t k = 0; k < U; k++)
                    n_cand += t2 + k * stride < n;
            uint32_t qq[U];
#pragma unroll
            for (uint32_t k = 0; k < U; k++) {
                qq[k] = 0;
                if (ww[k]) {
                    const uint64_t u = pc_div_small_q(X, mm[k]);
                    if (u < lo || u >= hi) { // cannot happen if the m range is right
                        atomicOr(A.err, 2);
                        ww[k] = 0;
                    } else {
                        qq[k] = (uint32_t)((u - lo + 1) >> 1);
                    }
                }
            }
#pragma unroll
            for (uint32_t k = 0; k < U; k++)
                if (ww[k]) {
                    lsum += (int64_t)ww[k] * (int64_t)(use_fen ? count_fen(qq[k]) : count_pre(qq[k]));
                    wsum += ww[k];
                    nleaf++;
                }
        }
        acc_local += lsum;
        return wsum;
    };
    // cross p_b of column j, items t0, t0 + stride, ... of its multiples, on
    // the exact current state; returns the integers this thread removed
    auto cross_exact = [&](uint32_t j, uint32_t t0, uint32_t stride) -> uint32_t {
        const uint32_t i0 = c_i0[j];
        uint32_t mine = 0;
        if (i0 < S) {
            const uint32_t p = c_p[j];
            const uint32_t n = (S - 1 - i0) / p + 1;
            for (uint32_t t2 = t0; t2 < n; t2 += stride) {
                const uint32_t bit = i0 + t2 * p;
                const uint32_t w = bit >> 5, mask = 1u << (bit & 31);
                if (BW(w) & mask) { // only this lane touches this bit
                    mine++;
                    fen_dec(bit >> BL);
                    __hip_atomic_fetch_and(&BW(w), ~mask, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
        return mine;
    };

    const uint32_t col_lo = tile.col_lo, col_hi = tile.col_hi;
    const uint32_t ncross = min(col_hi, Q.nb);
    for (uint32_t cb = 0; cb < ncross; cb += CH) {
        const uint32_t jend = min((uint32_t)CH, ncross - cb);
        if (tid == 0)
            s_first_large = jend;
        __syncthreads();
        // --- phase A: one lane per column: first multiple, leaf range ---
        bool leafy = false, heavy = false, large = false;
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
            large = (pc_u128)p * p * p >= hi;
            uint32_t ls = 0, lc = 0;
            if (MODE != PC_MODE_COUNT && col >= col_lo && col < col_hi) {
                const ulonglong2 ub = Q.Ub[b]; // u range of every hard leaf of b
                if (ub.x < hi && ub.y >= lo)
                    pc_leaf_range(TB, Q, b, p, rp, lo, hi, rhi, rlo, &ls, &lc);
            }
            c_ls[j] = ls;
            c_lc[j] = lc;
            c_new[j] = 0;
            c_w[j] = 0;
            leafy = lc != 0;
            heavy = (lc & ~PC_CAND) > LIGHT;
        }
        {
            const uint64_t bl = __ballot(leafy), bh = __ballot(heavy), bg = __ballot(large);
            if (lane == 0) {
                c_leafy[tid >> 6] = bl;
                c_heavy[tid >> 6] = bh;
                if (bg)
                    atomicMin(&s_first_large, (tid & ~63u) + (uint32_t)__builtin_ctzll(bg));
            }
        }
        __syncthreads();
        const uint32_t first_large = BATCH ? s_first_large : jend;
        uint32_t j = 0;

        // --- small primes (p^3 < hi): each thread crosses the words of the
        // blocks it owns, in prime order; no atomics and no barriers ---
        const uint32_t own0 = tid * OWN;
        for (; j < min(first_large, jend); j++) {
            const bool lf = (c_leafy[j >> 6] >> (j & 63)) & 1;
            if (lf) {
                n_leafy++;
                __syncthreads(); // every thread has crossed the columns before j
                build_pre();
                const uint32_t ws = pc_wave_sum_u32((uint32_t)leaves(cb, j, false, tid, T));
                if (lane == 0 && ws != 0)
                    atomicAdd(&c_w[j], (int32_t)ws);
                __syncthreads();
                if (MODE == PC_MODE_LEAVES && tid == 0)
                    acc_carry += (pc_s128)c_w[j] * (pc_s128)A.carry[row * ncol + cb + j];
            }
            const uint32_t i0 = c_i0[j];
            uint32_t mine = 0;
            if (i0 < S) {
                const uint32_t p = c_p[j];
                uint32_t f;
                if (i0 >= own0) {
                    f = i0;
                } else { // first multiple at or above own0: (own0 - i0) mod p by fp32 reciprocal
                    const uint32_t d = own0 - i0;
                    uint32_t q = (uint32_t)((float)d * __builtin_amdgcn_rcpf((float)p));
                    int32_t r = (int32_t)(d - q * p);
                    if (r < 0)
                        r += (int32_t)p;
                    else if (r >= (int32_t)p)
                        r -= (int32_t)p;
                    f = own0 + (r ? p - (uint32_t)r : 0);
                }
                for (uint32_t bit = f; bit < own0 + OWN; bit += p) {
                    const uint32_t w = bit >> 5, mask = 1u << (bit & 31);
                    const uint32_t v = BW(w);
                    if (v & mask) {
                        BW(w) = v & ~mask;
                        mine++;
                    }
                }
            }
            mine = pc_wave_sum_u32(mine);
            if (lane == 0 && mine)
                atomicAdd(&c_new[j], mine);
        }

        // --- large primes (p^3 >= hi), with the Fenwick tree ---
        if (j < jend) {
            if (!fen_ok) {
                __syncthreads(); // every thread has finished its small primes
                build_pre();
                build_fen();
                fen_ok = true;
            }
            while (j < jend) {
                const bool lf = (c_leafy[j >> 6] >> (j & 63)) & 1;
                const bool hv = (c_heavy[j >> 6] >> (j & 63)) & 1;
                if (lf && hv) {
                    // many leaves: the whole workgroup answers them, then crosses p_b
                    n_leafy++;
                    const uint32_t ws = pc_wave_sum_u32((uint32_t)leaves(cb, j, true, tid, T));
                    if (lane == 0 && ws != 0)
                        atomicAdd(&c_w[j], (int32_t)ws);
                    __syncthreads(); // leaf reads done before the column is crossed
                    if (MODE == PC_MODE_LEAVES && tid == 0)
                        acc_carry += (pc_s128)c_w[j] * (pc_s128)A.carry[row * ncol + cb + j];
                    const uint32_t mine = pc_wave_sum_u32(cross_exact(j, tid, T));
                    if (lane == 0 && mine)
                        atomicAdd(&c_new[j], mine);
                    __syncthreads();
                    j++;
                } else if (lf) {
                    // a run of light columns: wavefront 0 answers each column's
                    // leaves and crosses its prime in order, with no workgroup
                    // barrier; the run ends at a heavy column, at GAP leafless
                    // columns in a row, or at the chunk end
                    uint32_t jr = jend;
                    {
                        const uint32_t nwd = (jend + 63) / 64;
                        for (uint32_t wv = j >> 6; wv < nwd; wv++) {
                            const uint64_t keep = wv == (j >> 6) ? (~0ull << (j & 63)) : ~0ull;
                            const uint64_t z = ~c_leafy[wv];
                            uint64_t gap = z;
#pragma unroll
                            for (uint32_t g = 1; g < GAP; g++)
                                gap &= z >> g;
                            const uint64_t stop = (c_heavy[wv] | gap) & keep;
                            if (stop) {
                                jr = min(jend, wv * 64 + (uint32_t)__builtin_ctzll(stop));
                                break;
                            }
                        }
                    }
                    if (tid < 64) {
                        for (uint32_t jj = j; jj < jr; jj++) {
                            if ((c_leafy[jj >> 6] >> (jj & 63)) & 1) {
                                n_leafy++;
                                const uint32_t ws = pc_wave_sum_u32((uint32_t)leaves(cb, jj, true, lane, 64));
                                if (lane == 0) {
                                    c_w[jj] = (int32_t)ws;
                                    if (MODE == PC_MODE_LEAVES)
                                        acc_carry += (pc_s128)(int32_t)ws *
                                                     (pc_s128)A.carry[row * ncol + cb + jj];
                                }
                            }
                            const uint32_t mine = pc_wave_sum_u32(cross_exact(jj, lane, 64));
                            if (lane == 0)
                                c_new[jj] = mine;
                        }
                    }
                    __syncthreads();
                    j = jr;
                } else {
                    // run of leafless columns [j, jb), one lane per prime: an
                    // integer n = p k unsieved at the start of the run is first
                    // removed by p exactly when k = 1 or k >= p
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
                        uint32_t credit = 0;
                        const uint64_t p2 = (uint64_t)p * p;
                        for (uint32_t bit = i0; bit < S; bit += p)
                            if ((BW(bit >> 5) >> (bit & 31)) & 1) {
                                const uint64_t nn = lo + 2ull * bit + 1;
                                if (nn == p || nn >= p2) {
                                    credit++;
                                    fen_dec(bit >> BL);
                                }
                            }
                        c_new[jj] = credit;
                    }
                    __syncthreads(); // every read of the run precedes every clear
                    if (mine_col)
                        for (uint32_t bit = i0; bit < S; bit += p)
                            __hip_atomic_fetch_and(&BW(bit >> 5), ~(1u << (bit & 31)),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __syncthreads();
                    j = jb;
                }
            }
        } else {
            __syncthreads(); // c_new complete
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
        if (!fen_ok) {
            __syncthreads();
            build_pre();
        }
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
                acc_p2 += fen_ok ? count_fen(q) : count_pre(q);
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
#undef BW
    if (MODE != PC_MODE_COUNT) {
        const pc_s128 h = pc_block_sum128<T>((pc_s128)acc_local + acc_carry, scr128);
        const pc_s128 q = pc_block_sum128<T>((pc_s128)acc_p2 + extra_p2, scr128);
        nleaf = pc_wave_sum(nleaf);
        if (lane == 0 && nleaf)
            atomicAdd(&Q.sums->n_hard, nleaf);
        if (A.trace) {
            const uint32_t nc = pc_wave_sum_u32(n_cand);
            if (lane == 0) {
                atomicAdd(&A.trace[blockIdx.x].y, (uint32_t)nleaf);
                atomicAdd(&A.trace[blockIdx.x].z, nc);
            }
            __syncthreads();
            if (tid == 0) {
                A.trace[blockIdx.x].w = n_leafy;
                A.trace[blockIdx.x].x = (uint32_t)(__builtin_amdgcn_s_memrealtime() - t_start);
            }
        }
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

// ---------------------------------------------------------------------------
// Tile planning.  k_seg_work: hard-leaf items (primes m, or candidate m) that
// segment seg0 + blockIdx.x will answer, summed over every column.
// k_seg_split: for segment hot[i].x cut into hot[i].y tiles of about equal
// leaf work, the column boundaries (hot[i].y + 1 of them) at bounds[off_i].
// ---------------------------------------------------------------------------
#define PL_T 256

template <int LOG2_S>
__device__ __forceinline__ uint32_t pc_col_items(const pc_tables &TB, const pc_query &Q,
                                                 uint32_t col, uint64_t lo, uint64_t hi,
                                                 uint64_t rhi, uint64_t rlo)
{
    const uint32_t b = Q.c + 1 + col;
    const uint64_t p = TB.primes[b];
    uint32_t ls, lc;
    pc_leaf_range(TB, Q, b, p, TB.recip[b], lo, hi, rhi, rlo, &ls, &lc);
    return lc & ~PC_CAND;
}

template <int LOG2_S>
__global__ __launch_bounds__(PL_T) void k_seg_work(pc_tables TB, pc_query Q, uint64_t seg0,
                                                   uint64_t lo_base, uint64_t seg_base,
                                                   uint64_t *work)
{
    __shared__ uint64_t scr[PL_T / 64];
    const uint64_t seg = seg0 + blockIdx.x;
    const uint64_t lo = lo_base + ((seg - seg_base) << (LOG2_S + 1)), hi = lo + (2ull << LOG2_S);
    const uint64_t rhi = pc_recip(hi), rlo = lo ? pc_recip(lo) : 0;
    uint64_t s = 0;
    for (uint32_t col = threadIdx.x; col < Q.nb; col += PL_T)
        s += pc_col_items<LOG2_S>(TB, Q, col, lo, hi, rhi, rlo);
    s = pc_block_sum<PL_T>(s, scr);
    if (threadIdx.x == 0)
        work[blockIdx.x] = s;
}

template <int LOG2_S>
__global__ __launch_bounds__(PL_T) void k_seg_split(pc_tables TB, pc_query Q, const uint4 *hot,
                                                    uint64_t lo_base, uint64_t seg_base,
                                                    uint32_t *bounds)
{
    __shared__ uint64_t scr[PL_T / 64];
    const uint4 h = hot[blockIdx.x]; // x = segment, y = tiles K, z = offset, w = unused
    const uint64_t seg = h.x;
    const uint64_t lo = lo_base + ((seg - seg_base) << (LOG2_S + 1)), hi = lo + (2ull << LOG2_S);
    const uint64_t rhi = pc_recip(hi), rlo = lo ? pc_recip(lo) : 0;
    // total, then boundaries where the running work crosses j * total / K
    uint64_t tot = 0;
    for (uint32_t col = threadIdx.x; col < Q.nb; col += PL_T)
        tot += pc_col_items<LOG2_S>(TB, Q, col, lo, hi, rhi, rlo);
    tot = pc_block_sum<PL_T>(tot, scr);
    const uint64_t K = h.y;
    uint32_t *bd = bounds + h.z;
    if (threadIdx.x == 0) {
        bd[0] = 0;
        bd[K] = Q.ncol;
    }
    uint64_t run = 0;
    for (uint32_t c0 = 0; c0 < Q.nb; c0 += PL_T) {
        const uint32_t col = c0 + threadIdx.x;
        const uint64_t v = col < Q.nb ? pc_col_items<LOG2_S>(TB, Q, col, lo, hi, rhi, rlo) : 0;
        uint64_t chunk;
        const uint64_t e = run + pc_block_excl_scan<PL_T>(v, scr, &chunk);
        // tile j >= 1 starts at the first column whose exclusive prefix reaches j*tot/K
        if (col < Q.nb && tot > 0) {
            const uint64_t i = e + v;
            uint64_t j0 = (e * K) / tot + 1;     // smallest j with j*tot > e*K ... candidates
            for (uint64_t j = j0; j < K && j * tot <= i * K; j++)
                bd[j] = col + 1;
        }
        run += chunk;
    }
}

hipError_t pc_launch_seg_work(const pc_tables &T, const pc_query &Q, uint32_t seg_log2,
                              uint64_t lo_base, uint64_t seg_base, uint64_t seg0, uint32_t nseg,
                              uint64_t *work, hipStream_t s)
{
    if (nseg == 0)
        return hipSuccess;
    switch (seg_log2) {
    case 15: k_seg_work<15><<<nseg, PL_T, 0, s>>>(T, Q, seg0, lo_base, seg_base, work); break;
    case 16: k_seg_work<16><<<nseg, PL_T, 0, s>>>(T, Q, seg0, lo_base, seg_base, work); break;
    case 17: k_seg_work<17><<<nseg, PL_T, 0, s>>>(T, Q, seg0, lo_base, seg_base, work); break;
    case 18: k_seg_work<18><<<nseg, PL_T, 0, s>>>(T, Q, seg0, lo_base, seg_base, work); break;
    case 19: k_seg_work<19><<<nseg, PL_T, 0, s>>>(T, Q, seg0, lo_base, seg_base, work); break;
    case 20: k_seg_work<20><<<nseg, PL_T, 0, s>>>(T, Q, seg0, lo_base, seg_base, work); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t pc_launch_seg_split(const pc_tables &T, const pc_query &Q, uint32_t seg_log2,
                               uint64_t lo_base, uint64_t seg_base, const uint4 *hot,
                               uint32_t nhot, uint32_t *bounds, hipStream_t s)
{
    if (nhot == 0)
        return hipSuccess;
    switch (seg_log2) {
    case 15: k_seg_split<15><<<nhot, PL_T, 0, s>>>(T, Q, hot, lo_base, seg_base, bounds); break;
    case 16: k_seg_split<16><<<nhot, PL_T, 0, s>>>(T, Q, hot, lo_base, seg_base, bounds); break;
    case 17: k_seg_split<17><<<nhot, PL_T, 0, s>>>(T, Q, hot, lo_base, seg_base, bounds); break;
    case 18: k_seg_split<18><<<nhot, PL_T, 0, s>>>(T, Q, hot, lo_base, seg_base, bounds); break;
    case 19: k_seg_split<19><<<nhot, PL_T, 0, s>>>(T, Q, hot, lo_base, seg_base, bounds); break;
    case 20: k_seg_split<20><<<nhot, PL_T, 0, s>>>(T, Q, hot, lo_base, seg_base, bounds); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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
    // one-wavefront segments for the leaf-dense low end of [1, z]
    if (seg_log2 == 15 && wg == 64)
        return launch_modes<15, 64, 64>(A, mode, batch, s);
    if (seg_log2 == 16 && wg == 64)
        return launch_modes<16, 64, 64>(A, mode, batch, s);
    if (seg_log2 == 16 && wg == 128)
        return launch_modes<16, 128, 128>(A, mode, batch, s);
    if (seg_log2 == 17 && wg == 256)
        return launch_modes<17, 256, 256>(A, mode, batch, s);
    if (seg_log2 == 18 && wg == 256)
        return launch_modes<18, 256, 256>(A, mode, batch, s);
    if (seg_log2 == 18 && wg == 512)
        return launch_modes<18, 512, 512>(A, mode, batch, s);
    if (seg_log2 == 19 && wg == 512)
        return launch_modes<19, 512, 512>(A, mode, batch, s);
    if (seg_log2 == 19 && wg == 1024)
        return launch_modes<19, 1024, 1024>(A, mode, batch, s);
    return hipErrorInvalidValue;
}

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
// >= p) each wave crosses up to 64 columns of its region in one step, one
// lane per prime: an integer n = p k unsieved at the start of the step is
// first removed by p exactly when k = 1 or k >= p, which gives the
// per-column counts without ordering the lanes.
#include "pc_block.h"
#include "pc_internal.h"
#include "pc_leafrange.h"

// PC_PHASE_TRACE=1 adds per-phase tick counters to the tile trace (a
// profiling build; the default build only records totals)
#ifndef PC_PHASE_TRACE
#define PC_PHASE_TRACE 0
#endif


// Waves per SIMD that the LDS footprint of k_sieve<LOG2_S, T, CH> allows on a
// CU (160 KiB of LDS, at most 8 waves per SIMD); the kernel asks the compiler
// to fit its registers to that many, so a code change cannot silently cost a
// resident workgroup.
template <int LOG2_S, int T, int CH> constexpr uint32_t pc_sieve_gcap()
{
    return (1u << (LOG2_S - 9)) > 256u ? (1u << (LOG2_S - 9)) : 256u;
}
template <int LOG2_S, int T, int CH> constexpr int pc_sieve_waves_per_simd()
{
    constexpr long S = 1l << LOG2_S, NW = S / 32, NWP = NW + NW / 16, NBLK = S >> 9;
    constexpr long NWV = T / 64;
    constexpr long KMAX = 64; // gathered columns per round (g_rc, g_rm)
    constexpr long lds = 4 * (NWP + 16) + 4 * (NBLK + 1) + 4 * pc_sieve_gcap<LOG2_S, T, CH>() +
                         2 * KMAX * NWV + 8 * KMAX + 24 * CH + 16 * (CH / 64) + 8 + 8 * NWV +
                         16 * NWV;
    constexpr long wg = 163840 / lds;
    constexpr long waves = wg * NWV < 32 ? wg * NWV : 32;
    return waves / 4 < 1 ? 1 : (int)(waves / 4);
}

template <int LOG2_S, int T, int CH, int MODE, bool BATCH>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(
    pc_sieve_waves_per_simd<LOG2_S, T, CH>()))) void k_sieve(pc_sieve_args A)
{
    static_assert(CH == T, "one lane per column of a chunk");
    static_assert(T % 64 == 0, "wavefront multiples");
    constexpr uint32_t S = 1u << LOG2_S;   // odd integers (bits) per segment
    constexpr uint32_t NW = S / 32;        // 32-bit words
    constexpr uint32_t NWP = NW + NW / 16; // padded: one spare word after every 16
    constexpr uint32_t BL = 9;             // 512-bit counting blocks (16 words)
    constexpr uint32_t NBLK = S >> BL;
    constexpr uint32_t NWV = T / 64;
    constexpr uint32_t BPT = NBLK / T; // counting blocks per thread
    static_assert(NBLK % T == 0 && BPT >= 1 && BPT <= 2, "every thread counts one or two blocks");
    constexpr uint32_t RS = S / NWV;   // bits of the region a wavefront owns
    constexpr uint32_t RSL = LOG2_S - (NWV == 1 ? 0 : NWV == 2 ? 1 : NWV == 4 ? 2 : NWV == 8 ? 3 : 4);
    static_assert((1u << RSL) == RS && RS == 64 * BPT * 512, "a region is 64 threads' blocks");
    constexpr uint32_t GCAP = pc_sieve_gcap<LOG2_S, T, CH>(); // gathered leaf items
    constexpr uint32_t LIGHT = GCAP / 4; // more leaf items: the column is answered workgroup-wide
    constexpr uint32_t XB_P = RS / 32;   // p >= XB_P: at most 32 multiples in a wave's region
    constexpr uint32_t KMAX = 64;         // columns per gather round (as in pc_sieve_waves_per_simd)
    static_assert(GCAP < 2048 && LIGHT < 2048, "gathered-column fields");
    static_assert(GCAP >= 64 * NWV, "64 slots of gbuf per wave in a heavy column");

    // Word w of the segment lives at bm[w + w/16]: the 16 words of a counting
    // block are contiguous and consecutive blocks start 17 words apart, so the
    // threads of a wavefront walking their own blocks hit distinct banks.
    __shared__ uint32_t bm[NWP + 16];  // 16 spare words: a query at q = S reads past the end
    __shared__ uint32_t pre[NBLK + 1]; // prefix of the block counts; or a gather round's table
    __shared__ uint32_t gbuf[GCAP];    // gathered leaves: k << 22 | q << 2 | (mu(m) > 0) << 1 | 1
    __shared__ uint16_t g_rc[KMAX * NWV]; // each wave's region count at gathered column k
    __shared__ uint32_t g_rm[2 * KMAX];   // regions that hold a leaf of gathered column k (2 rounds)
    __shared__ uint32_t c_p[CH];       // p_b
    __shared__ uint32_t c_i0[CH];      // bit of the first multiple in the segment, S if none
    __shared__ uint32_t c_ls[CH];      // first leaf item (m, or index of the prime m)
    __shared__ uint32_t c_lc[CH];      // leaf items; PC_CAND: items are candidates (pc_wheel_m)
    __shared__ uint32_t c_new[CH];     // integers first removed by p_b in this segment
    __shared__ int32_t c_w[CH];        // sum of -mu(m) over the leaves of the column
    __shared__ uint64_t c_leafy[CH / 64];
    __shared__ uint64_t c_heavy[CH / 64];
    __shared__ uint32_t s_first_large, s_first_skip;
    __shared__ uint32_t scr32[NWV];
    __shared__ pc_s128 scr128[NWV];

    const uint64_t t_start = A.trace ? __builtin_amdgcn_s_memrealtime() : 0;
    uint32_t n_cand = 0, n_leafy = 0, n_leafy_small = 0;
#if PC_PHASE_TRACE
    // 0 set-up, 1 per-column set-up, 2 gathers, 3 heavy columns, 4 wavefront
    // columns, 5 batched crossings, 7 chunk results, 8 final column; event
    // counts: 0 column crossings by a wave, 1 answered columns, 2 gather rounds
    uint32_t ph[9] = {}, ev[3] = {};
    uint64_t ph_last = t_start;
#define PC_EV(k) (ev[k]++)
#define PC_PH(k)                                                                        \
    do {                                                                                \
        if (A.trace) {                                                                  \
            const uint64_t t_ = __builtin_amdgcn_s_memrealtime();                       \
            ph[k] += (uint32_t)(t_ - ph_last);                                          \
            ph_last = t_;                                                               \
        }                                                                               \
    } while (0)
#else
#define PC_PH(k) \
    do {         \
    } while (0)
#define PC_EV(k) ((void)0)
#endif
    pc_tile tile = A.tiles[blockIdx.x];
    tile.seg = pc_uniform(tile.seg);
    tile.col_lo = pc_uniform(tile.col_lo);
    tile.col_hi = pc_uniform(tile.col_hi);
    tile.q = pc_uniform(tile.q);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    if (tile.col_lo >= tile.col_hi) { // a split that owns no column
        if (MODE != PC_MODE_COUNT && tid == 0 && A.part_hard) {
            A.part_hard[blockIdx.x] = 0;
            A.part_p2[blockIdx.x] = 0;
        }
        return;
    }
    const uint64_t seg = tile.seg;
    const uint64_t lo = A.lo_base + ((seg - A.seg_base) << (LOG2_S + 1));
    const uint64_t hi = lo + (2ull << LOG2_S);
    const uint64_t row = seg - A.seg0;
    const pc_query &Q = A.Qs[tile.q];
    // this row's cells of cnt / wgt: columns [0, r_len) from r_off on (a
    // bound on the columns that still have hard leaves at or above lo)
    const uint64_t r_off = Q.row_off ? pc_uniform64(Q.row_off[row]) : row * Q.nb;
    const uint32_t r_len =
        Q.row_off ? pc_uniform((uint32_t)(Q.row_off[row + 1] - Q.row_off[row])) : Q.nb;
    const uint32_t qc = pc_uniform(Q.c);
    const uint64_t *const Xb1 = pc_uniform_ptr(Q.Xb) + qc + 1; // X_b of column j of chunk cb: Xb1[cb + j]
    // above 2^64 the leaf quotients take X_b's value in fp64 beside its low word
    const bool wide = Q.x_hi != 0;
    const double *const Xd1 = Q.Xd + qc + 1;
    const pc_tables &TB = A.T;
    const uint64_t rhi = pc_recip(hi);
    const uint64_t rlo = lo ? pc_recip(lo) : 0;
    const uint32_t ncol = Q.ncol;
#define BW(w) bm[(w) + ((w) >> 4)]

    // --- pre-sieved state: the wheel pattern (p_2..p_c already crossed) ---
    {
        const uint32_t P = TB.pattern_bits;
        const uint32_t g0 = (uint32_t)((lo >> 1) % P);
        const uint32_t step = (32u * T) % P; // from word w to word w + T
        uint32_t off = (uint32_t)(((uint64_t)g0 + 32u * tid) % P);
        for (uint32_t w = tid; w < NW; w += T) {
            const uint32_t wi = off >> 5, sh = off & 31;
            uint32_t v = TB.pattern[wi] >> sh;
            if (sh)
                v |= TB.pattern[wi + 1] << (32 - sh);
            BW(w) = v;
            off += step;
            if (off >= P)
                off -= P;
        }
    }
    if (tid < 2 * KMAX)
        g_rm[tid] = 0;
    __syncthreads();

    // unsieved integers in each of the blocks thread tid counts
    auto block_counts = [&](uint32_t (&cnt)[BPT]) -> uint32_t {
        uint32_t s = 0;
#pragma unroll
        for (uint32_t k = 0; k < BPT; k++) {
            const uint32_t base = (tid * BPT + k) * 17;
            uint32_t c = 0;
#pragma unroll
            for (uint32_t i = 0; i < 16; i++)
                c += (uint32_t)__builtin_popcount(bm[base + i]);
            cnt[k] = c;
            s += c;
        }
        return s;
    };
    // pre[] = exclusive prefix of the unsieved counts of the blocks; returns
    // the segment total.  Every thread must call it; it ends with a barrier.
    auto build_pre = [&]() -> uint32_t {
        uint32_t cnt[BPT];
        const uint32_t s = block_counts(cnt);
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
    // unsieved integers of q's block on q's side: below q when q lies in the
    // block's lower half (*up false), at or above q otherwise; eight words
    auto half_count = [&](uint32_t q, bool *up) -> uint32_t {
        const uint32_t nw = (q >> 5) & 15, part = (1u << (q & 31)) - 1;
        *up = nw >= 8;
        const uint32_t base = (q >> BL) * 17 + (*up ? 8u : 0u), k0 = *up ? 8u : 0u;
        const uint32_t below = *up ? 0u : ~0u, at = *up ? ~part : part, above = ~below;
        uint32_t s = 0;
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            const uint32_t m = k0 + k < nw ? below : (k0 + k == nw ? at : above);
            s += (uint32_t)__builtin_popcount(bm[base + k] & m);
        }
        return s;
    };
    // unsieved integers among bits [0, q), q <= S, against pre[]
    auto count_pre = [&](uint32_t q) -> uint32_t {
        bool up;
        const uint32_t s = half_count(q, &up), blk = q >> BL;
        return up ? pre[blk + 1] - s : pre[blk] + s;
    };
    // A wave's own blocks with finer sums (one block per thread): the block's
    // unsieved count, and in *pk the prefix counts of its first one, two and
    // three quarters of 128 bits (10 bits each).
    auto block_counts_q = [&](uint32_t *pk) -> uint32_t {
        const uint32_t base = tid * 17;
        uint32_t qs[4];
#pragma unroll
        for (uint32_t k = 0; k < 4; k++) {
            uint32_t c = 0;
#pragma unroll
            for (uint32_t i = 0; i < 4; i++)
                c += (uint32_t)__builtin_popcount(bm[base + 4 * k + i]);
            qs[k] = c;
        }
        const uint32_t p1 = qs[0], p2 = p1 + qs[1], p3 = p2 + qs[2];
        *pk = p1 | (p2 << 10) | (p3 << 20);
        return p3 + qs[3];
    };
    // unsieved integers of q's block below q, from the block's quarter
    // prefixes pk and total tb: two words of q's quarter are read, the ones
    // on q's side (up from the quarter's start, or down from its end)
    auto quarter_count = [&](uint32_t q, uint32_t pk, uint32_t tb) -> uint32_t {
        const uint32_t off = q & 511u, qq = off >> 7, w = (off >> 5) & 3u;
        const uint32_t part = (1u << (q & 31u)) - 1u; // bits below q in its word
        const uint32_t below = qq ? (pk >> (10u * (qq - 1u))) & 1023u : 0u;
        const uint32_t through = qq < 3u ? (pk >> (10u * qq)) & 1023u : tb;
        const bool low = w < 2u;
        const uint32_t a0 = (q >> BL) * 17u + qq * 4u + (low ? 0u : 2u);
        const uint32_t v0 = bm[a0], v1 = bm[a0 + 1];
        if (low) // words [0, w) of the quarter and the part of w below q
            return below + (uint32_t)__builtin_popcount(v0 & (w == 0u ? part : ~0u)) +
                   (uint32_t)__builtin_popcount(v1 & (w == 1u ? part : 0u));
        // the quarter less the rest of w and the words after it
        return through - (uint32_t)__builtin_popcount(v0 & (w == 2u ? ~part : 0u)) -
               (uint32_t)__builtin_popcount(v1 & (w == 2u ? ~0u : ~part));
    };

    uint32_t total = build_pre();
    PC_PH(0);
    // Wavefront wv owns bits [R0, R1).  rc = its unsieved integers, kept exact
    // through every crossing: a leaf whose u lies in a higher region counts
    // all of them, one in this region counts a prefix of it.
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));
    const uint32_t R0 = wv * RS, R1 = R0 + RS;
    uint32_t rc = (uint32_t)__builtin_amdgcn_readfirstlane((int)(pre[R1 >> BL] - pre[R0 >> BL]));
    unsigned long long nleaf = 0;      // hard leaves answered by this thread
    int64_t acc_local = 0;             // sum of -mu(m) * in-segment count (hard leaves)
    int64_t acc_p2 = 0;                // sum of in-segment counts (P2 terms)
    pc_s128 acc_carry = 0;             // PC_MODE_LEAVES: carry * w
    uint32_t g_par = 0;                // g_rm half of the current gather round

    // Leaf item it of column j: *m and *w = -mu(m), false if the candidate m
    // is not squarefree with lpf(m) > p_b.
    auto leaf_filter = [&](uint32_t j, uint32_t it, uint64_t *m, int32_t *w) -> bool {
        const uint32_t lc = c_lc[j], ls = c_ls[j];
        if (lc & PC_CAND) {
            const uint32_t mc = pc_wheel_m(TB, ls + it);
            const int32_t v = TB.mulpf[mc];
            const uint32_t av = v < 0 ? (uint32_t)(-v) : (uint32_t)v;
            n_cand++;
            *m = mc;
            *w = v > 0 ? -1 : 1;
            return av > c_p[j];
        }
        *m = TB.primes[ls + it];
        *w = 1;
        return true;
    };
    // q = bits of the segment below u = floor(X_b / m), u in [lo, hi); X is
    // X_b modulo 2^64 and Xd its value in fp64 (read only above 2^64)
    auto leaf_q = [&](uint64_t X, double Xd, uint64_t m, bool *ok) -> uint32_t {
        const uint64_t u = wide ? pc_div_small_qd(X, Xd, (uint32_t)m) : pc_div_small_q(X, m);
        *ok = u >= lo && u < hi;
        if (!*ok) // cannot happen if the m range is right
            atomicOr(A.err, 2);
        return (uint32_t)((u - lo + 1) >> 1);
    };

    const uint32_t col_lo = tile.col_lo, col_hi = tile.col_hi;
    const uint32_t ncross = min(col_hi, Q.nb);
    bool recounted = false; // the carried count was checked against the bitmap (uniform)
    for (uint32_t cb = 0; cb < ncross; cb += CH) {
        const uint32_t jall = min((uint32_t)CH, ncross - cb);
        if (tid == 0) {
            s_first_large = jall;
            s_first_skip = jall;
        }
        __syncthreads();
        // --- one lane per column: first multiple, leaf range ---
        bool leafy = false, heavy = false, large = false, skip = false;
        if (tid < jall) {
            const uint32_t j = tid, col = cb + j, b = qc + 1 + col;
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
            // every hard leaf of b and of the later primes lies below ub.y
            const ulonglong2 ub = Q.Ub[b];
            skip = ub.y < lo;
            if (MODE != PC_MODE_COUNT && col >= col_lo && col < col_hi && ub.x < hi && !skip)
                pc_leaf_range(TB, Q, b, p, rp, lo, hi, rhi, rlo, &ls, &lc);
            c_ls[j] = ls;
            c_lc[j] = lc;
            c_new[j] = 0;
            c_w[j] = 0;
            leafy = lc != 0;
            heavy = (lc & ~PC_CAND) > LIGHT;
        }
        {
            const uint64_t bl = __ballot(leafy), bh = __ballot(heavy), bg = __ballot(large);
            const uint64_t bs = __ballot(skip);
            if (lane == 0) {
                c_leafy[tid >> 6] = bl;
                c_heavy[tid >> 6] = bh;
                if (bg)
                    atomicMin(&s_first_large, (tid & ~63u) + (uint32_t)__builtin_ctzll(bg));
                if (bs)
                    atomicMin(&s_first_skip, (tid & ~63u) + (uint32_t)__builtin_ctzll(bs));
            }
        }
        __syncthreads();
        PC_PH(1);
        // columns [jend, jall) and every later chunk's are past their last hard
        // leaf (skip, a suffix): they are only cleared, after this chunk
        const uint32_t jend = s_first_skip;
        const uint32_t first_large = BATCH ? min(s_first_large, jend) : jend;

        // For 64 columns from cg0 on (one column per lane): p, the first
        // multiple of p at or above R0 and the number of its multiples in
        // [R0, R1), computed together; v_rem collects each column's removals
        // in its lane and goes to c_new once per 64 columns.
        uint32_t cg0 = 0x80000000u, v_f = 0, v_p = 1, v_nm = 0, v_rem = 0; // j - cg0 >= 64: reload
        auto flush_removed = [&]() {
            if (v_rem)
                atomicAdd(&c_new[cg0 + lane], v_rem);
            v_rem = 0;
        };
        // the group of 64 columns that holds column j
        auto ensure_group = [&](uint32_t j) {
            if (j - cg0 >= 64) {
                flush_removed();
                cg0 = j;
                v_p = 1;
                v_nm = 0;
                v_f = 0;
                if (j + lane < jend) {
                    const uint32_t i0 = c_i0[j + lane], p = c_p[j + lane];
                    // floor(e / p) for e < 2^20: the fp32 reciprocal puts the
                    // estimate within one of the quotient, one step corrects it
                    const float rp = __builtin_amdgcn_rcpf((float)p);
                    auto quot = [&](uint32_t e) -> uint32_t {
                        uint32_t q = (uint32_t)((float)e * rp);
                        const int32_t r = (int32_t)(e - q * p);
                        if (r < 0)
                            q--;
                        else if (r >= (int32_t)p)
                            q++;
                        return q;
                    };
                    uint32_t f = i0;
                    if (i0 < R0) {
                        const uint32_t d = R0 - i0, r = d - quot(d) * p;
                        f = R0 + (r ? p - r : 0);
                    }
                    v_p = p;
                    v_f = f;
                    v_nm = f < R1 ? quot(R1 - 1 - f) + 1 : 0;
                }
            }
        };
        // cross column cg0 + k, which has nm > 0 multiples in this wave's
        // region, one lane per multiple
        auto cross_k = [&](int32_t k, uint32_t nm) {
            PC_EV(0);
            const uint32_t f = (uint32_t)__builtin_amdgcn_readlane((int)v_f, k);
            const uint32_t p = (uint32_t)__builtin_amdgcn_readlane((int)v_p, k);
            // a lane's multiples lie 64 p bits apart, a multiple of 32: they
            // all sit at the same bit of their words, 2 p words apart
            const uint32_t bit = f + lane * p;
            const uint32_t sh = bit & 31, keep = ~(1u << sh), wstep = 2 * p;
            uint32_t w = bit >> 5;
            auto clear = [&](uint32_t wd) -> uint32_t {
                const uint32_t old = __hip_atomic_fetch_and(&BW(wd), keep, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
                return (old >> sh) & 1u;
            };
            uint32_t removed = 0;
            const uint32_t full = nm >> 6; // rounds in which every lane has a multiple
            if (full) {
                uint32_t hits = 0, t = 0;
                for (; t + 2 <= full; t += 2, w += 2 * wstep) // two clears in flight
                    hits += clear(w) + clear(w + wstep);
                if (t < full) {
                    hits += clear(w);
                    w += wstep;
                }
                removed = pc_wave_sum_u32(hits);
            }
            bool hit = false;
            if (lane < (nm & 63))
                hit = clear(w) != 0;
            removed += (uint32_t)__builtin_popcountll(__ballot(hit));
            rc -= removed;
            if (lane == (uint32_t)k)
                v_rem = removed;
        };
        auto cross_region = [&](uint32_t j) {
            ensure_group(j);
            const int32_t k = (int32_t)(j - cg0);
            const uint32_t nm = (uint32_t)__builtin_amdgcn_readlane((int)v_nm, k);
            if (nm)
                cross_k(k, nm);
        };
        // Large columns [ja, jb) of the cached group (every one at or past
        // first_large, with p >= XB_P) crossed in this wave's region in one
        // step, one lane per column.  An integer n = p k unsieved at the start
        // is first removed by p exactly when k = 1 or k >= p (p^3 >= hi leaves
        // n at most two prime factors, none below the first column's prime),
        // so each lane first reads its multiples and credits those, then
        // clears them; the order of the columns no longer matters.  Gathered
        // leaves in slots [es0, es1) that lie in this region are answered in
        // between: their count at the start, less the credited multiples
        // below them of the earlier columns.
        auto xbatch = [&](uint32_t ja, uint32_t jb, uint32_t es0, uint32_t es1) {
            const uint32_t col = cg0 + lane;
            const uint32_t nm = col >= ja && col < jb ? v_nm : 0u;
            const uint32_t f = v_f, p = v_p;
            // n = lo + 2 bit + 1 >= p^2  <=>  bit >= tb;  n = p  <=>  bit = ip
            const uint64_t p2 = (uint64_t)p * p;
            const uint32_t tb = p2 <= lo ? 0u : (uint32_t)min<uint64_t>(S, (p2 - lo - 1) >> 1);
            const uint32_t ip = lo <= p ? (uint32_t)((p - lo - 1) >> 1) : S;
            uint32_t cm = 0; // credited multiples: bit i <-> f + i p
            for (uint32_t i = 0; __ballot(i < nm); i++)
                if (i < nm) {
                    const uint32_t bit = f + i * p;
                    if (((BW(bit >> 5) >> (bit & 31)) & 1u) && (bit >= tb || bit == ip))
                        cm |= 1u << i;
                }
            if (es0 < es1) {
                bool have = false;
                uint32_t pe = 0, pc0 = 0, pq = 0; // lane prefix of the region's block counts;
                // first block (or, one block a lane, its count and quarter prefixes)
                const float rp = __builtin_amdgcn_rcpf((float)p);
                for (uint32_t s = es0; s < es1; s += 64) {
                    const uint32_t e = s + lane < es1 ? gbuf[s + lane] : 0u;
                    const uint32_t q = (e >> 2) & 0xFFFFFu;
                    const bool in = (e & 1) && (q >> RSL) == wv;
                    uint64_t pend = __ballot(in);
                    if (!pend)
                        continue;
                    if (!have) {
                        uint32_t sum;
                        if (BPT > 1) {
                            uint32_t cnt[BPT];
                            sum = block_counts(cnt);
                            pc0 = cnt[0];
                        } else {
                            sum = block_counts_q(&pq);
                            pc0 = sum;
                        }
                        pe = pc_wave_incl_scan_u32(sum) - sum;
                        have = true;
                    }
                    const uint32_t bl = in ? (q >> BL) - (R0 >> BL) : 0u;
                    const uint32_t src = bl / BPT;
                    uint32_t c = (uint32_t)__shfl((int)pe, (int)src, 64);
                    if (BPT > 1) {
                        const uint32_t c0 = (uint32_t)__shfl((int)pc0, (int)src, 64);
                        c += (bl % BPT) ? c0 : 0u;
                        if (in)
                            c += in_block(q);
                    } else { // the block is its lane's: count from its quarter prefixes
                        const uint32_t tb = (uint32_t)__shfl((int)pc0, (int)src, 64);
                        const uint32_t pk = (uint32_t)__shfl((int)pq, (int)src, 64);
                        if (in)
                            c += quarter_count(q, pk, tb);
                    }
                    // less the earlier columns' credited multiples below q:
                    // leaf by leaf (all lanes count for one leaf) or column
                    // by column (all leaves count one column), the shorter
                    uint64_t cols = __ballot(cm != 0);
                    if (__builtin_popcountll(pend) <= __builtin_popcountll(cols)) {
                        while (pend) {
                            const int32_t l = (int32_t)__builtin_ctzll(pend);
                            pend &= pend - 1;
                            const uint32_t ql = (uint32_t)__builtin_amdgcn_readlane((int)q, l);
                            const uint32_t kl = (uint32_t)__builtin_amdgcn_readlane((int)e, l) >> 22;
                            uint32_t below = 0;
                            if (lane < kl && cm != 0 && ql > f) {
                                const uint32_t d = ql - f - 1; // multiples f + t p, t <= d / p
                                uint32_t t = (uint32_t)((float)d * rp);
                                const int32_t r = (int32_t)(d - t * p);
                                if (r < 0)
                                    t--;
                                else if (r >= (int32_t)p)
                                    t++;
                                below = (uint32_t)__builtin_popcount(t >= 31 ? cm : cm & ((2u << t) - 1));
                            }
                            const uint32_t tot = pc_wave_sum_u32(below);
                            if (lane == (uint32_t)l)
                                c -= tot;
                        }
                    } else {
                        const uint32_t ke = e >> 22;
                        while (cols) {
                            const int32_t k = (int32_t)__builtin_ctzll(cols);
                            cols &= cols - 1;
                            const uint32_t fk = (uint32_t)__builtin_amdgcn_readlane((int)f, k);
                            const uint32_t pk = (uint32_t)__builtin_amdgcn_readlane((int)p, k);
                            const uint32_t ck = (uint32_t)__builtin_amdgcn_readlane((int)cm, k);
                            if (in && ke > (uint32_t)k && q > fk) {
                                const uint32_t d = q - fk - 1;
                                uint32_t t = (uint32_t)((float)d * __builtin_amdgcn_rcpf((float)pk));
                                const int32_t r = (int32_t)(d - t * pk);
                                if (r < 0)
                                    t--;
                                else if (r >= (int32_t)pk)
                                    t++;
                                c -= (uint32_t)__builtin_popcount(t >= 31 ? ck : ck & ((2u << t) - 1));
                            }
                        }
                    }
                    if (in)
                        acc_local += (e & 2) ? -(int64_t)c : (int64_t)c;
                }
            }
            for (uint32_t i = 0; __ballot(i < nm); i++)
                if (i < nm) {
                    const uint32_t bit = f + i * p;
                    __hip_atomic_fetch_and(&BW(bit >> 5), ~(1u << (bit & 31)), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            const uint32_t cr = (uint32_t)__builtin_popcount(cm);
            if (nm)
                v_rem = cr;
            rc -= pc_wave_sum_u32(cr);
        };
        // the first column of [j, je) (within the cached group) from which on
        // xbatch applies, or je
        auto xbatch_from = [&](uint32_t j, uint32_t je) -> uint32_t {
            if (!BATCH)
                return je;
            const uint32_t col = cg0 + lane;
            const uint64_t lg = __ballot(col >= j && col < je && col >= first_large && v_p >= XB_P);
            return lg ? cg0 + (uint32_t)__builtin_ctzll(lg) : je;
        };
        // cross the leafless columns [j, je) in this wave's region, visiting
        // only those with a multiple in it
        auto cross_run = [&](uint32_t j, uint32_t je) {
            while (j < je) {
                ensure_group(j);
                const uint32_t ge = min(je, cg0 + 64);
                const uint32_t xb = xbatch_from(j, ge);
                uint64_t msk = __ballot(v_nm != 0 && cg0 + lane >= j && cg0 + lane < xb);
                while (msk) {
                    const int32_t k = (int32_t)__builtin_ctzll(msk);
                    msk &= msk - 1;
                    cross_k(k, (uint32_t)__builtin_amdgcn_readlane((int)v_nm, k));
                }
                if (xb < ge)
                    xbatch(xb, ge, 0, 0);
                j = ge;
            }
        };

        // Gather rounds.  The leaves of the light leafy columns of a window
        // (whole columns of one cached group of 64, in order, stopping at the
        // next heavy column or when GCAP slots are full) go to gbuf, one
        // candidate per slot; column cg0 + k is the round's column k.  Each
        // wave answers only the leaves whose u lies in its own region, and
        // records its region count per column in g_rc; when the round is over
        // (every wave past its columns), settle() adds, for every leaf, the
        // counts of the regions below its own.  Every wave computes the
        // round's slot offsets itself, and thread t only ever reads and writes
        // slots t, t + T, ..., so a round needs two barriers.
        uint32_t g_used = 0; // slots of the open round (uniform); 0 = none open
        auto settle = [&]() { // after a barrier that every wave reached past the round
            for (uint32_t s = tid; s < g_used; s += T) {
                const uint32_t e = gbuf[s];
                if (!(e & 1))
                    continue;
                const uint32_t k = e >> 22, r = min(((e >> 2) & 0xFFFFFu) >> RSL, NWV);
                uint32_t below = 0;
                for (uint32_t w = 0; w < r; w++)
                    below += g_rc[k * NWV + w];
                acc_local += (e & 2) ? -(int64_t)below : (int64_t)below;
            }
            g_used = 0;
        };
        // j0 lies in the cached group and we <= cg0 + 64; returns the end of
        // the round's window: every light leafy column of [j0, that end) is
        // gathered, and pre[k] = slot offset << 11 | items of column cg0 + k
        // (0 for columns outside the round or without leaves).
        auto gather = [&](uint32_t j0, uint32_t we) -> uint32_t {
            PC_PH(4);
            __syncthreads(); // every wave is past the open round's columns
            settle();
            PC_EV(2);
            g_par ^= 1;
            // the next heavy column at or after j0 ends the round
            uint32_t hvn = jend;
            {
                uint32_t wd = j0 >> 6;
                uint64_t msk = c_heavy[wd] & (~0ull << (j0 & 63));
                while (!msk && ++wd < (jend + 63) / 64)
                    msk = c_heavy[wd];
                if (msk)
                    hvn = min(jend, wd * 64 + (uint32_t)__builtin_ctzll(msk));
            }
            hvn = min(hvn, we);
            const uint32_t col = cg0 + lane;
            uint32_t v = 0;
            if (col >= j0 && col < hvn)
                v = c_lc[col] & ~PC_CAND; // light: heavy columns lie at or past hvn
            const uint32_t inc = pc_wave_incl_scan_u32(v), off = inc - v;
            const uint64_t over = __ballot(v != 0 && inc > GCAP);
            const uint32_t kend = over ? (uint32_t)__builtin_ctzll(over) : 64u;
            const uint32_t used = kend ? (uint32_t)__builtin_amdgcn_readlane((int)off, (int)(kend - 1)) +
                                             (uint32_t)__builtin_amdgcn_readlane((int)v, (int)(kend - 1))
                                       : 0u;
            uint32_t *const rm = g_rm + g_par * KMAX;
            if (tid < KMAX)
                g_rm[(g_par ^ 1) * KMAX + tid] = 0; // the next round's masks
            for (uint32_t s0 = 0; s0 < used; s0 += T) {
                // the column of slot s: the last lane whose offset is <= s
                const uint32_t s = s0 + tid;
                uint32_t a = 0, oa = 0;
#pragma unroll
                for (uint32_t h = 32; h; h >>= 1) {
                    const uint32_t o = (uint32_t)__shfl((int)off, (int)(a + h), 64);
                    if (o <= s) {
                        a += h;
                        oa = o;
                    }
                }
                int32_t wl = 0;   // -mu(m) of this slot's leaf, 0 if none
                uint32_t rl = 0xFFu; // its region (0xFF: none, or above every region)
                if (s < used) {
                    const uint32_t aj = cg0 + a;
                    uint64_t m;
                    int32_t w;
                    uint32_t e = 0;
                    if (leaf_filter(aj, s - oa, &m, &w)) {
                        bool ok;
                        const uint32_t q =
                            leaf_q(Xb1[cb + aj], wide ? Xd1[cb + aj] : 0.0, m, &ok);
                        if (ok) {
                            const uint32_t r = q >> RSL;
                            e = (a << 22) | (q << 2) | (w < 0 ? 2u : 0u) | 1u;
                            wl = w;
                            rl = r < NWV ? r : 0xFFu;
                            nleaf++;
                        }
                    }
                    gbuf[s] = e;
                }
                // The wave's slots are consecutive, so its lanes hold runs of one
                // column (and within a column, of one region: u falls with m).
                // Column weights: one add per run, from a wave scan of the
                // weights; region masks: one OR per run of (column, region).
                const uint32_t key = s < used ? a : 0xFFu;
                const uint32_t kr = key << 8 | rl;
                const uint32_t kr_prev = (uint32_t)__shfl_up((int)kr, 1, 64);
                if (rl != 0xFFu && (lane == 0 || kr_prev != kr))
                    atomicOr(&rm[a], 1u << rl);
                const uint32_t inc = pc_wave_incl_scan_u32((uint32_t)wl);
                const uint32_t key_next = (uint32_t)__shfl_down((int)key, 1, 64);
                const bool tail = lane == 63 || key_next != key;
                const uint64_t below = __ballot(tail) & ((1ull << lane) - 1);
                const int32_t pt = below ? 63 - __builtin_clzll(below) : 0;
                const uint32_t base = (uint32_t)__shfl((int)inc, pt, 64);
                const int32_t run = (int32_t)(inc - (below ? base : 0u));
                if (tail && key != 0xFFu && run != 0)
                    atomicAdd(&c_w[cg0 + key], run);
            }
            if (wv == 0) { // the round's table
                const bool g = lane < kend && v != 0;
                pre[lane] = g ? (off << 11) | v : 0u;
                n_leafy += g ? 1u : 0u;
                n_leafy_small += g && col < first_large ? 1u : 0u;
            }
            g_used = used;
            __syncthreads();
            PC_PH(2);
            return over ? min(hvn, cg0 + kend) : hvn;
        };
        // this wave's part of the leaves of gathered column j that lie in its
        // region: a prefix of the region for each
        auto answer = [&](uint32_t g) {
            PC_EV(1);
            const uint32_t s0 = g >> 11, s1 = s0 + (g & 0x7FFu);
            bool have = false;
            uint32_t pe = 0, pc0 = 0, pq = 0; // lane prefix of the region's block counts;
                // first block (or, one block a lane, its count and quarter prefixes)
            for (uint32_t s = s0; s < s1; s += 64) {
                const uint32_t e = s + lane < s1 ? gbuf[s + lane] : 0u;
                const uint32_t q = (e >> 2) & 0xFFFFFu;
                const bool in = (e & 1) && (q >> RSL) == wv;
                if (__ballot(in)) {
                    if (!have) {
                        uint32_t sum;
                        if (BPT > 1) {
                            uint32_t cnt[BPT];
                            sum = block_counts(cnt);
                            pc0 = cnt[0];
                        } else {
                            sum = block_counts_q(&pq);
                            pc0 = sum;
                        }
                        pe = pc_wave_incl_scan_u32(sum) - sum;
                        have = true;
                    }
                    const uint32_t bl = in ? (q >> BL) - (R0 >> BL) : 0u;
                    const uint32_t src = bl / BPT;
                    uint32_t c = (uint32_t)__shfl((int)pe, (int)src, 64);
                    if (BPT > 1) {
                        const uint32_t c0 = (uint32_t)__shfl((int)pc0, (int)src, 64);
                        c += (bl % BPT) ? c0 : 0u;
                    }
                    const uint32_t tb = (uint32_t)__shfl((int)pc0, (int)src, 64);
                    const uint32_t pk = (uint32_t)__shfl((int)pq, (int)src, 64);
                    if (in) {
                        if (BPT > 1)
                            c += in_block(q);
                        else // the block is its lane's: count from its quarter prefixes
                            c += quarter_count(q, pk, tb);
                        acc_local += (e & 2) ? -(int64_t)c : (int64_t)c;
                    }
                }
            }
        };
        // Many leaves: the whole workgroup answers them against pre[].  Prime
        // items are all leaves (each thread loads HU of them before it divides);
        // each wave filters its own candidates, HU * 64 loads at a time, and
        // packs the survivors into its 64 slots of gbuf, so the divisions and
        // counts run on full wavefronts without workgroup barriers.
        auto heavy_col = [&](uint32_t j) {
            constexpr uint32_t HU = 2;
            PC_PH(4);
            __syncthreads(); // every wave has crossed the columns before j
            settle();
            build_pre();     // (its barriers also end settle's reads of gbuf)
            const uint32_t lc = c_lc[j], n = lc & ~PC_CAND, ls = c_ls[j];
            const uint64_t X = pc_uniform64(Xb1[cb + j]);
            const double Xd = wide ? Xd1[cb + j] : 0.0;
            int32_t wsum = 0;
            int64_t lsum = 0;
            auto one = [&](uint64_t m, int32_t w) {
                bool ok;
                const uint32_t q = leaf_q(X, Xd, m, &ok);
                if (ok) {
                    lsum += (int64_t)w * (int64_t)count_pre(q);
                    wsum += w;
                    nleaf++;
                }
            };
            if (!(lc & PC_CAND)) {
                for (uint32_t it0 = tid; it0 < n; it0 += HU * T) {
                    uint32_t mm[HU];
#pragma unroll
                    for (uint32_t u = 0; u < HU; u++)
                        mm[u] = it0 + u * T < n ? TB.primes[ls + it0 + u * T] : 0u;
#pragma unroll
                    for (uint32_t u = 0; u < HU; u++)
                        if (it0 + u * T < n)
                            one(mm[u], 1);
                }
            } else {
                const uint32_t p = c_p[j];
                uint32_t *const slot = gbuf + wv * 64; // this wave's slots
                uint32_t held = 0;                     // filled slots (uniform)
                // slot entry: m | (mu(m) > 0) << 31
                auto drain = [&]() {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    if (lane < held) {
                        const uint32_t e = slot[lane];
                        one(e & 0x7FFFFFFFu, (e >> 31) ? -1 : 1);
                    }
                    held = 0;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                };
                // the loop bound is uniform: drain() needs every lane of the wave
                for (uint32_t base = wv * 64 * HU; base < n; base += HU * T) {
                    const uint32_t it0 = base + lane;
                    int32_t v[HU];
                    uint32_t mm[HU];
#pragma unroll
                    for (uint32_t u = 0; u < HU; u++) {
                        mm[u] = pc_wheel_m(TB, ls + it0 + u * 64);
                        v[u] = it0 + u * 64 < n ? TB.mulpf[mm[u]] : 0;
                    }
#pragma unroll
                    for (uint32_t u = 0; u < HU; u++) {
                        const uint32_t it = it0 + u * 64;
                        n_cand += it < n ? 1u : 0u;
                        const uint32_t av = v[u] < 0 ? (uint32_t)(-v[u]) : (uint32_t)v[u];
                        const bool keep = av > p; // squarefree (v != 0), lpf(m) > p_b
                        const uint64_t bal = __ballot(keep);
                        const uint32_t k = (uint32_t)__builtin_popcountll(bal);
                        if (held + k > 64)
                            drain();
                        if (keep)
                            slot[held + (uint32_t)__builtin_popcountll(bal & ((1ull << lane) - 1))] =
                                mm[u] | (v[u] > 0 ? 0x80000000u : 0u);
                        held += k;
                        if (held == 64)
                            drain();
                    }
                }
                if (held)
                    drain();
            }
            acc_local += lsum;
            const uint32_t ws = pc_wave_sum_u32((uint32_t)wsum);
            if (lane == 0 && ws != 0)
                atomicAdd(&c_w[j], (int32_t)ws);
            if (tid == 0) {
                n_leafy++;
                if (j < first_large)
                    n_leafy_small++;
            }
            __syncthreads(); // every read of the column's state precedes its crossing
            PC_PH(3);
        };
        // Columns [j, we) of one cached group, their light leaves gathered:
        // each wave visits, in order, the columns that have a leaf in its
        // region (answered before the crossing) or a multiple in it, then
        // records its region count before each gathered column (its count at
        // j minus the removals of the window's earlier columns).
        auto window = [&](uint32_t j, uint32_t we) {
            const uint32_t rc0 = rc;
            const uint32_t col = cg0 + lane;
            const bool inw = col >= j && col < we;
            const uint32_t xb = xbatch_from(j, we); // columns from xb on: one xbatch step
            const bool sm = col < xb;
            const uint32_t g = inw ? pre[lane] : 0u; // the round's table
            const bool gath = g != 0;
            const uint32_t rm = gath ? g_rm[g_par * KMAX + lane] : 0u;
            const bool mine = gath && ((rm >> wv) & 1u);
            const uint64_t own = __ballot(mine && sm);
            const uint64_t crs = __ballot(inw && sm && v_nm != 0);
            uint64_t todo = own | crs;
            while (todo) {
                const int32_t k = (int32_t)__builtin_ctzll(todo);
                todo &= todo - 1;
                if ((own >> k) & 1)
                    answer((uint32_t)__builtin_amdgcn_readlane((int)g, k));
                if ((crs >> k) & 1)
                    cross_k(k, (uint32_t)__builtin_amdgcn_readlane((int)v_nm, k));
            }
            if (xb < we) {
                // the large columns' slots run from the first one gathered to
                // the end of the round
                const uint64_t gl = __ballot(mine && !sm);
                const uint32_t es0 =
                    gl ? (uint32_t)__builtin_amdgcn_readlane((int)g, (int)__builtin_ctzll(gl)) >> 11
                       : g_used;
                xbatch(xb, we, es0, g_used);
            }
            const uint32_t rem = inw ? v_rem : 0u;
            const uint32_t before = pc_wave_incl_scan_u32(rem) - rem;
            if (gath)
                g_rc[lane * NWV + wv] = (uint16_t)(rc0 - before);
        };
        // Columns in order.  Each wave crosses its own region, so between the
        // workgroup-wide steps (gather, heavy column) the waves move through
        // the columns independently.
        uint32_t j = 0, jb_next = 0; // jb_next: the next leafy column, once known
        uint32_t lw_at = ~0u;        // c_leafy word cached for columns [64 lw_at, 64 lw_at + 64)
        uint64_t lw = 0;
        while (j < jend) {
            if ((j >> 6) != lw_at) {
                lw_at = j >> 6;
                lw = c_leafy[lw_at];
            }
            if ((lw >> (j & 63)) & 1) { // leaves, then the crossing
                const bool hv = (c_heavy[j >> 6] >> (j & 63)) & 1;
                if (hv) {
                    heavy_col(j);
                    cross_region(j);
                    j++;
                } else { // a window within j's group of 64 columns
                    ensure_group(j);
                    const uint32_t we = gather(j, min(jend, cg0 + 64));
                    window(j, we);
                    j = we;
                }
                continue;
            }
            if (jb_next <= j) { // the next leafy column after j
                uint32_t wd = j >> 6;
                uint64_t msk = c_leafy[wd] & (~0ull << (j & 63));
                while (!msk && ++wd < (jend + 63) / 64)
                    msk = c_leafy[wd];
                jb_next = msk ? min(jend, wd * 64 + (uint32_t)__builtin_ctzll(msk)) : jend;
            }
            // a leafless run, each wave in its own region (large primes a
            // group of 64 at a time, xbatch)
            cross_run(j, jb_next);
            j = jb_next;
        }
        flush_removed();
        PC_PH(4);
        __syncthreads(); // c_new complete; every wave is past the open round
        settle();
        // --- chunk results: cnt before each crossing, and w ---
        {
            const uint32_t v = tid < jend ? c_new[tid] : 0;
            uint32_t tot;
            const uint32_t ex = pc_block_excl_scan<T>(v, scr32, &tot);
            const uint32_t col = cb + tid;
            // columns at or past the cut hold no leaf here or below: 0 (if stored)
            if (tid < jall && col < r_len && col >= col_lo && col < col_hi) {
                const bool cut = tid >= jend;
                const uint64_t idx = r_off + col;
                if (MODE != PC_MODE_LEAVES)
                    Q.cnt[idx] = cut ? 0u : total - ex;
                if (MODE == PC_MODE_TALLY)
                    Q.wgt[idx] = cut ? 0 : c_w[tid];
                if (MODE == PC_MODE_LEAVES && !cut && c_w[tid] != 0)
                    acc_carry += (pc_s128)c_w[tid] * (pc_s128)Q.carry[idx];
            }
            // every column before the cut must be stored: the row's bound holds
            if (tid < jend && col >= r_len && col >= col_lo && col < col_hi)
                atomicOr(A.err, 8);
            total -= tot;
        }
        PC_PH(7);
        if (jend < jall) {
            // Device invariant: the unsieved count carried through every
            // crossing so far (each wave's own hits, summed per column) must
            // equal a fresh count of the bitmap.
            if (build_pre() != total && tid == 0)
                atomicOr(A.err, 32);
            recounted = true;
            // Every column from cb + jend on is past its last hard leaf: its
            // count is read by no leaf and it removes nothing a later leaf of
            // this segment counts, so its multiples are only cleared, in any
            // order, one thread per column.  Its stored counts are 0.
            for (uint32_t col = cb + jend + tid; col < ncross; col += T) {
                const uint32_t b = qc + 1 + col;
                const uint64_t p = TB.primes[b];
                uint64_t first = p;
                if (lo > p) {
                    first = pc_div(lo, p, TB.recip[b]) * p;
                    if (first < lo)
                        first += p;
                    if ((first & 1) == 0)
                        first += p;
                }
                if (first < hi)
                    for (uint32_t bit = (uint32_t)((first - lo - 1) >> 1); bit < S; bit += (uint32_t)p)
                        __hip_atomic_fetch_and(&BW(bit >> 5), ~(1u << (bit & 31)), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                if (MODE != PC_MODE_LEAVES && col >= cb + jall && col < r_len && col >= col_lo &&
                    col < col_hi) {
                    Q.cnt[r_off + col] = 0;
                    if (MODE == PC_MODE_TALLY)
                        Q.wgt[r_off + col] = 0;
                }
            }
            PC_PH(5);
            break;
        }
    }

    // --- final column: P2 lookups pi(x/p) = phi(x/p, bmax) + bmax - 1 ---
    pc_s128 extra_p2 = 0; // PC_MODE_LEAVES: carry * (lookups), kept by thread 0
    if (col_hi == ncol) {
        __syncthreads();
        const uint32_t rec = build_pre(); // (the carried total skips the cleared-only columns)
        if (!recounted && rec != total && tid == 0)
            atomicOr(A.err, 32); // the invariant above, for a segment with no cut
        total = rec;
        uint32_t k1 = 1, k2 = 0;
        {
            // x/p < hi <=> p > x/hi;  x/p >= lo <=> p <= x/lo  (above 2^64: every
            // segment but the first has lo >= 2^16, so both quotients are < 2^52)
            const uint64_t tA = Q.x_hi ? pc_div_wide(Q.x, Q.xd, hi) : pc_div(Q.x, hi, rhi);
            const uint64_t tB =
                !lo ? ~0ull : Q.x_hi ? pc_div_wide(Q.x, Q.xd, lo) : pc_div(Q.x, lo, rlo);
            const uint64_t pl = tA > Q.y ? tA : Q.y;
            const uint64_t ph = tB < Q.sqrtx ? tB : Q.sqrtx;
            if (pl < ph) {
                k1 = pc_pi_lookup(TB.pitab, pl) + 1;
                k2 = pc_pi_lookup(TB.pitab, ph);
            }
        }
        if (MODE != PC_MODE_COUNT) {
            const uint64_t x = Q.x;     // modulo 2^64 above 2^64
            const double xd = Q.xd;
            for (uint32_t k = k1 + tid; k <= k2; k += T) {
                uint32_t off; // x/p_k - lo
                const bool in = k < TB.k32
                                    ? pc_quot_in(x, xd, TB.primes[k], lo, 2u << LOG2_S, &off)
                                    : pc_quot_in64(x, xd, TB.primes_hi[k - TB.k32], lo,
                                                   2u << LOG2_S, &off);
                if (!in) {
                    atomicOr(A.err, 4);
                    continue;
                }
                acc_p2 += count_pre((off + 1) >> 1);
            }
        }
        if (tid == 0) {
            const uint32_t np = k2 >= k1 ? k2 - k1 + 1 : 0;
            if (MODE != PC_MODE_LEAVES)
                Q.cntP[row] = total;
            if (MODE == PC_MODE_TALLY)
                Q.wP[row] = (int32_t)np;
            if (MODE == PC_MODE_LEAVES)
                extra_p2 = (pc_s128)np * (pc_s128)Q.carryP[row];
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
            uint32_t *tr = A.trace + (size_t)blockIdx.x * PC_TRACE_W;
            const uint32_t nc = pc_wave_sum_u32(n_cand);
            const uint32_t nl = pc_wave_sum_u32(n_leafy);
            const uint32_t ns = pc_wave_sum_u32(n_leafy_small);
            if (lane == 0) {
                atomicAdd(&tr[1], (uint32_t)nleaf);
                atomicAdd(&tr[2], nc);
                atomicAdd(&tr[3], nl);
                atomicAdd(&tr[4], ns);
            }
            __syncthreads();
            PC_PH(8);
            if (tid == 0) {
                tr[0] = (uint32_t)(__builtin_amdgcn_s_memrealtime() - t_start);
#if PC_PHASE_TRACE
                for (int k = 0; k < 9; k++)
                    tr[5 + k] = ph[k];
                tr[11] = ev[0]; // phase 6 is unused
                tr[14] = ev[1];
                tr[15] = ev[2];
#endif
            }
        }
        if (tid == 0) {
            if (A.part_hard) {
                A.part_hard[blockIdx.x] = h;
                A.part_p2[blockIdx.x] = q;
            } else {
                pc_atomic_add128(&Q.sums->hard_local, h);
                pc_atomic_add128(&Q.sums->p2_local, q);
            }
        }
    }
}
#undef PC_PH
#undef PC_EV

// ---------------------------------------------------------------------------
// Look-back scan over the segments of a window, independently per column:
// carry[s][col] = carry_in[col] + sum_{s' < s} cnt[s'][col], over the rows
// that store the column (a prefix of the window's rows: row lengths never
// grow).  Workgroups take tickets in order; ticket t is block t - blkoff[k]
// of chunk k (256 columns by rows_per_chunk rows).  A workgroup publishes
// its column sums and looks back through earlier chunks until one has
// published an inclusive prefix (decoupled look-back); a column stored in a
// chunk's first row is stored in every earlier chunk, so every look-back
// finds its words.
//
// PC_MODE_TALLY needs only sum w * carry, which splits over a chunk as
//   sum_r w_r (P + l_r) = P * sum_r w_r + sum_r w_r l_r,
// P = the carry at the chunk's first row (from the look-back), l_r = the
// counts of the chunk's rows above r: one pass over cnt and wgt before the
// look-back, each read once, SCAN_U rows of loads in flight per thread.
// PC_MODE_COUNT writes every carry out for the leaf pass (a second pass).
// ---------------------------------------------------------------------------
#define SCAN_T 256
#define SCAN_U 8
#define SCAN_RMAX 1024
#define LB_A (1ull << 62)
#define LB_P (2ull << 62)
#define LB_V ((1ull << 62) - 1)

template <int MODE> __global__ __launch_bounds__(SCAN_T) void k_scan(pc_scan_args A)
{
    __shared__ uint32_t s_ticket, s_chunk;
    __shared__ uint64_t s_off[SCAN_RMAX + 1];
    __shared__ pc_s128 scr[SCAN_T / 64];
    if (threadIdx.x == 0) {
        const uint32_t t = atomicAdd(A.ticket, 1u);
        uint32_t lo = 0, hi = A.nchunk - 1; // the chunk k with blkoff[k] <= t < blkoff[k+1]
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (A.blkoff[mid] <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        s_ticket = t;
        s_chunk = lo;
    }
    __syncthreads();
    const uint32_t tk = s_ticket, rc = s_chunk;
    const uint32_t cb = tk - A.blkoff[rc];
    const uint64_t r0 = (uint64_t)rc * A.rows_per_chunk;
    const uint32_t nr = (uint32_t)min<uint64_t>(A.rows_per_chunk, A.nrows - r0);
    for (uint32_t i = threadIdx.x; i <= nr; i += SCAN_T)
        s_off[i] = A.row_off[r0 + i];
    __syncthreads();
    const uint32_t col = cb * SCAN_T + threadIdx.x;
    // rows of the chunk that store the column: a prefix [0, na)
    uint32_t na = 0;
    {
        uint32_t lo = 0, hi = nr; // the first row whose length is <= col
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_off[mid + 1] - s_off[mid] > col)
                lo = mid + 1;
            else
                hi = mid;
        }
        na = lo;
    }
    const bool act = na > 0;
    uint64_t agg = 0, pre = 0;
    int64_t wsum = 0;   // PC_MODE_TALLY: sum of w over the chunk
    pc_s128 wl = 0;     //                sum of w * (counts of the chunk above the row)
    if (act) {
        if (MODE == PC_MODE_TALLY) {
            uint32_t i = 0;
            for (; i + SCAN_U <= na; i += SCAN_U) {
                uint32_t c[SCAN_U];
                int32_t w[SCAN_U];
#pragma unroll
                for (uint32_t u = 0; u < SCAN_U; u++) {
                    c[u] = A.cnt[s_off[i + u] + col];
                    w[u] = A.wgt[s_off[i + u] + col];
                }
#pragma unroll
                for (uint32_t u = 0; u < SCAN_U; u++) {
                    if (w[u]) {
                        wsum += w[u];
                        wl += (pc_s128)((int64_t)w[u] * (int64_t)agg);
                    }
                    agg += c[u];
                }
            }
            for (; i < na; i++) {
                const int32_t w = A.wgt[s_off[i] + col];
                if (w) {
                    wsum += w;
                    wl += (pc_s128)((int64_t)w * (int64_t)agg);
                }
                agg += A.cnt[s_off[i] + col];
            }
        } else {
            for (uint32_t i = 0; i < na; i++)
                agg += A.cnt[s_off[i] + col];
        }
        // look-back words: one per (ticket, thread); chunk rc - 1 holds this
        // column in its block cb
        uint64_t *st = A.status + (uint64_t)tk * SCAN_T + threadIdx.x;
        if (rc == 0) {
            __hip_atomic_store(st, LB_P | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(st, LB_A | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t jc = (int64_t)rc - 1;
            uint32_t spins = 0;
            while (jc >= 0) {
                const uint64_t w = ((uint64_t)A.blkoff[jc] + cb) * SCAN_T + threadIdx.x;
                const uint64_t v =
                    __hip_atomic_load(A.status + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    pc_s128 dh = 0;
    if (act) {
        const uint64_t P = A.carry_in[col] + pre; // carry at the chunk's first row
        if (MODE == PC_MODE_TALLY) {
            dh = (pc_s128)wsum * (pc_s128)P + wl;
        } else {
            uint64_t carry = P;
            for (uint32_t i = 0; i < na; i++) {
                A.carry_rows[s_off[i] + col] = carry;
                carry += A.cnt[s_off[i] + col];
            }
        }
        // a column stored through the window's last row continues in the next window
        if (rc == A.nchunk - 1 && na == nr)
            A.carry_out[col] = P + agg;
    }
    if (MODE == PC_MODE_TALLY) {
        dh = pc_block_sum128<SCAN_T>(dh, scr);
        if (threadIdx.x == 0)
            A.part_hard[tk] = dh;
    }
}

// The P2 column: carry = carry_in + sum of cntP over the rows above, and
// sum wP * carry (PC_MODE_TALLY) or every carry (PC_MODE_COUNT); one
// workgroup, each thread a run of consecutive rows.
#define SCANP_T 1024
template <int MODE> __global__ __launch_bounds__(SCANP_T) void k_scan_p2(pc_scan_args A)
{
    __shared__ uint64_t scr[SCANP_T / 64];
    __shared__ pc_s128 scr128[SCANP_T / 64];
    const uint64_t per = (A.nrows + SCANP_T - 1) / SCANP_T;
    const uint64_t r0 = min<uint64_t>(A.nrows, threadIdx.x * per), r1 = min(A.nrows, r0 + per);
    uint64_t agg = 0;
    for (uint64_t r = r0; r < r1; r++)
        agg += A.cntP[r];
    uint64_t tot;
    uint64_t carry = A.carry_in[A.nb] + pc_block_excl_scan<SCANP_T>(agg, scr, &tot);
    pc_s128 acc = 0;
    for (uint64_t r = r0; r < r1; r++) {
        if (MODE == PC_MODE_TALLY) {
            const int32_t w = A.wP[r];
            if (w)
                acc += (pc_s128)w * (pc_s128)carry;
        } else {
            A.carryP[r] = carry;
        }
        carry += A.cntP[r];
    }
    if (threadIdx.x == 0)
        A.carry_out[A.nb] = A.carry_in[A.nb] + tot;
    if (MODE == PC_MODE_TALLY) {
        acc = pc_block_sum128<SCANP_T>(acc, scr128);
        if (threadIdx.x == 0)
            *A.part_p2 = acc;
    }
}

hipError_t pc_launch_scan(const pc_scan_args &A, int mode, hipStream_t s)
{
    if (A.nrows == 0)
        return hipSuccess;
    if (A.rows_per_chunk == 0 || A.rows_per_chunk > SCAN_RMAX ||
        (uint64_t)A.nchunk * A.rows_per_chunk < A.nrows)
        return hipErrorInvalidValue;
    if (mode == PC_MODE_TALLY) {
        if (A.nticket)
            k_scan<PC_MODE_TALLY><<<A.nticket, SCAN_T, 0, s>>>(A);
        k_scan_p2<PC_MODE_TALLY><<<1, SCANP_T, 0, s>>>(A);
    } else {
        if (A.nticket)
            k_scan<PC_MODE_COUNT><<<A.nticket, SCAN_T, 0, s>>>(A);
        k_scan_p2<PC_MODE_COUNT><<<1, SCANP_T, 0, s>>>(A);
    }
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

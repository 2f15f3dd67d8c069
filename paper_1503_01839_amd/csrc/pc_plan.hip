// pc_plan.hip -- tile planning for the sieve: estimated leaf work per segment
// and column-range cuts of the hottest segments.
#include "pc_block.h"
#include "pc_internal.h"
#include "pc_leafrange.h"

// ---------------------------------------------------------------------------
// Tile planning.  k_seg_work: hard-leaf items (primes m, or candidate m) that
// segment seg0 + blockIdx.x will answer, summed over every column.
// k_seg_split: for segment hot[i].x cut into hot[i].y tiles of about equal
// leaf work, the column boundaries (hot[i].y + 1 of them) at bounds[off_i].
// ---------------------------------------------------------------------------
#define PL_T 256

// Estimated leaf work of column col in the segment [lo, hi), for balancing
// tiles only: candidates m (each read and tested), or about twice the number
// of primes m in range (each a leaf), without the pi-table reads.
template <int LOG2_S>
__device__ __forceinline__ uint32_t pc_col_items(const pc_tables &TB, const pc_query &Q,
                                                 uint32_t col, uint64_t lo, uint64_t hi,
                                                 uint64_t rhi, uint64_t rlo)
{
    const uint32_t b = Q.c + 1 + col;
    const ulonglong2 ub = Q.Ub[b];
    if (ub.x >= hi || ub.y < lo)
        return 0;
    const uint64_t p = TB.primes[b];
    uint64_t m1, m2;
    pc_leaf_mrange(Q, b, p, TB.recip[b], lo, hi, rhi, rlo, &m1, &m2);
    if (m1 > m2)
        return 0;
    const uint64_t n = m2 - m1 + 1;
    if (p <= Q.sqrty) // candidates prime to p_1..p_c
        return (uint32_t)((float)n * ((float)TB.phiQ / (float)TB.Qc)) + 1u;
    return (uint32_t)(2.0f * (float)n / __logf((float)m2 + 2.0f)) + 1u;
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


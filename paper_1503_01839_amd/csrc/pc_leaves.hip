// pc_leaves.hip -- one-query kernels for the parts of phi(x, a) = S1 + S2 that
// need no sieve (S1, trivial and easy special leaves) and the final
// combination; the per-item work is in pc_leafwork.h.
#include "pc_leafwork.h"

#define LV_T 256

// ---------------------------------------------------------------------------
// S1: one lane per n <= y (grid-stride).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LV_T) void k_s1(pc_tables T, pc_query Q, pc_s128 *part)
{
    __shared__ pc_s128 scr[LV_T / 64];
    __shared__ unsigned long long scr64[LV_T / 64];
    const uint32_t pcc = T.primes[Q.c];
    pc_s128 acc = 0;
    unsigned long long terms = 0;
    const uint64_t stride = (uint64_t)gridDim.x * LV_T;
    for (uint64_t n = 1 + (uint64_t)blockIdx.x * LV_T + threadIdx.x; n <= Q.y; n += stride)
        terms += pc_s1_item(T, Q, pcc, n, &acc);
    acc = pc_block_sum128<LV_T>(acc, scr);
    terms = pc_block_sum<LV_T>(terms, scr64);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc;
        atomicAdd(&Q.sums->n_s1, terms);
    }
}

hipError_t pc_launch_s1(const pc_tables &T, const pc_query &Q, pc_s128 *part, uint32_t nblocks,
                        hipStream_t s)
{
    k_s1<<<nblocks, LV_T, 0, s>>>(T, Q, part);
    return hipGetLastError();
}

// X_b for b <= a (pc_xb_item).
__global__ __launch_bounds__(LV_T) void k_xb(pc_tables T, pc_query Q)
{
    pc_xb_item(T, Q, blockIdx.x * LV_T + threadIdx.x);
}

hipError_t pc_launch_xb(const pc_tables &T, const pc_query &Q, hipStream_t s)
{
    k_xb<<<Q.a / LV_T + 1, LV_T, 0, s>>>(T, Q);
    return hipGetLastError();
}

// Per-b set-up of the special leaves outside the sieve (pc_leaf_setup_item).
__global__ __launch_bounds__(LV_T) void k_leaf_setup(pc_tables T, pc_query Q, pc_s128 *part_t)
{
    __shared__ uint64_t scr[LV_T / 64];
    uint64_t triv, cross;
    pc_leaf_setup_item(T, Q, blockIdx.x * LV_T + threadIdx.x, &triv, &cross);
    const uint64_t s = pc_block_sum<LV_T>(triv, scr);
    const uint64_t cs = pc_block_sum<LV_T>(cross, scr);
    if (threadIdx.x == 0) {
        part_t[blockIdx.x] = (pc_s128)s;
        atomicAdd(&Q.sums->n_trivial, (unsigned long long)s);
        atomicAdd(&Q.sums->crossings, (unsigned long long)cs);
    }
}

__global__ __launch_bounds__(1024) void k_ub_suffix(pc_query Q)
{
    __shared__ uint64_t sh[1024];
    pc_ub_suffix<1024>(Q, sh);
}

hipError_t pc_launch_leaf_setup(const pc_tables &T, const pc_query &Q, pc_s128 *part_trivial,
                                uint32_t nblocks, hipStream_t s)
{
    k_leaf_setup<<<nblocks, LV_T, 0, s>>>(T, Q, part_trivial);
    k_ub_suffix<<<1, 1024, 0, s>>>(Q);
    return hipGetLastError();
}

// e_off[b] = exclusive prefix of the item counts (mode bit stripped)
__global__ void k_strip_counts(const uint64_t *e_count, uint64_t *e_off, uint64_t n)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        e_off[i] = e_count[i] & ~PC_MODEBIT;
}

// Candidate easy leaves of one query, tiles of EZ_T * EZ_PER items (pc_easy_tiles).
#define EZ_T 256
#define EZ_PER 32

__global__ __launch_bounds__(EZ_T) void k_easy(pc_tables T, pc_query Q, pc_s128 *part)
{
    __shared__ pc_s128 scr[EZ_T / 64];
    __shared__ unsigned long long scr64[EZ_T / 64];
    __shared__ uint32_t s_b0;
    unsigned long long nleaf = 0;
    int64_t acc = 0;
    pc_easy_tiles<EZ_T, EZ_PER>(T, Q, blockIdx.x, gridDim.x, &s_b0, &acc, &nleaf);
    const pc_s128 s = pc_block_sum128<EZ_T>((pc_s128)acc, scr);
    nleaf = pc_block_sum<EZ_T>(nleaf, scr64);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s;
        atomicAdd(&Q.sums->n_easy, nleaf);
    }
}

hipError_t pc_launch_easy(const pc_tables &T, const pc_query &Q, pc_s128 *part, uint32_t nblocks,
                          hipStream_t s)
{
    k_easy<<<nblocks, EZ_T, 0, s>>>(T, Q, part);
    return hipGetLastError();
}

// The bands of the singles and groups (pc_easy_band_item), one thread per band.
__global__ __launch_bounds__(LV_T) void k_easy_bands(pc_tables T, pc_query Q)
{
    pc_easy_band_item(T, Q, blockIdx.x * LV_T + threadIdx.x);
}

hipError_t pc_launch_easy_bands(const pc_tables &T, const pc_query &Q, hipStream_t s)
{
    const uint32_t nband = Q.a / PC_EZ_BAND + 1;
    k_easy_bands<<<(nband + LV_T - 1) / LV_T, LV_T, 0, s>>>(T, Q);
    return hipGetLastError();
}

// The singles and the groups of the easy leaves of one query (pc_easy_bands).
__global__ __launch_bounds__(PC_EZ_UNIT) void k_easy_band(pc_tables T, pc_query Q, pc_s128 *part)
{
    __shared__ pc_s128 scr[PC_EZ_UNIT / 64];
    __shared__ uint32_t s_g[2];
    int64_t acc = 0;
    pc_easy_bands<PC_EZ_UNIT, false>(T, Q, blockIdx.x, gridDim.x, &s_g[0], &acc);
    pc_easy_bands<PC_EZ_UNIT, true>(T, Q, blockIdx.x, gridDim.x, &s_g[1], &acc);
    const pc_s128 s = pc_block_sum128<PC_EZ_UNIT>((pc_s128)acc, scr);
    if (threadIdx.x == 0)
        part[blockIdx.x] = s;
}

hipError_t pc_launch_easy_band(const pc_tables &T, const pc_query &Q, pc_s128 *part,
                               uint32_t nblocks, hipStream_t s)
{
    k_easy_band<<<nblocks, PC_EZ_UNIT, 0, s>>>(T, Q, part);
    return hipGetLastError();
}

hipError_t pc_launch_strip(const uint64_t *e_count, uint64_t *e_off, uint64_t n, hipStream_t s)
{
    k_strip_counts<<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(e_count, e_off, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// acc += sum of part[0..n)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LV_T) void k_sum128(const pc_s128 *part, uint32_t n, pc_s128 *acc)
{
    __shared__ pc_s128 scr[LV_T / 64];
    pc_s128 s = 0;
    for (uint32_t i = threadIdx.x; i < n; i += LV_T)
        s += part[i];
    s = pc_block_sum128<LV_T>(s, scr);
    if (threadIdx.x == 0)
        *acc += s;
}

hipError_t pc_launch_sum128(const pc_s128 *part, uint32_t n, pc_s128 *acc, hipStream_t s)
{
    k_sum128<<<1, LV_T, 0, s>>>(part, n, acc);
    return hipGetLastError();
}

__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = v;
}

hipError_t pc_launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    uint64_t nb = (n + 255) / 256;
    if (nb > 65536)
        nb = 65536;
    k_fill_u64<<<(uint32_t)nb, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

// pi(x) and its parts from the partial sums (pc_combine_one).
__global__ void k_combine(const pc_sums *S, pc_query Q, uint64_t kp2, pc_final *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        pc_combine_one(*S, Q, kp2, out);
}

hipError_t pc_launch_combine(const pc_sums *sums, const pc_query &Q, uint64_t kp2, pc_final *out,
                             hipStream_t s)
{
    k_combine<<<1, 64, 0, s>>>(sums, Q, kp2, out);
    return hipGetLastError();
}

// pc_batch.hip -- many pi(x) queries in one pass: the same per-item work as
// the one-query kernels (pc_leafwork.h) on flat grids whose blocks are dealt
// out to the queries by host-built tables, with every query's sums
// accumulated in place (pc_atomic_add128).  The sieve itself is the one-query
// kernel: its tiles name their query.
#include "pc_leafwork.h"

#define BT 256
#define BEZ_PER 32

// block -> (query, block of the query, blocks of the query)
struct pc_blk {
    const uint32_t *q;     // query of each block
    const uint32_t *first; // first block of each query; first[nq] = total
};

__device__ __forceinline__ void pc_blk_of(const pc_blk &B, uint32_t *q, uint32_t *lb,
                                          uint32_t *nlb)
{
    *q = B.q[blockIdx.x];
    const uint32_t f = B.first[*q];
    *lb = blockIdx.x - f;
    *nlb = B.first[*q + 1] - f;
}

__global__ __launch_bounds__(BT) void k_xb_b(pc_tables T, const pc_query *Qs, pc_blk B)
{
    uint32_t q, lb, nlb;
    pc_blk_of(B, &q, &lb, &nlb);
    const pc_query &Q = Qs[q];
    for (uint32_t b = lb * BT + threadIdx.x; b <= Q.a; b += nlb * BT)
        pc_xb_item(T, Q, b);
}

__global__ __launch_bounds__(BT) void k_s1_b(pc_tables T, const pc_query *Qs, pc_blk B)
{
    __shared__ pc_s128 scr[BT / 64];
    __shared__ unsigned long long scr64[BT / 64];
    uint32_t q, lb, nlb;
    pc_blk_of(B, &q, &lb, &nlb);
    const pc_query &Q = Qs[q];
    const uint32_t pcc = T.primes[Q.c];
    pc_s128 acc = 0;
    unsigned long long terms = 0;
    for (uint64_t n = 1 + (uint64_t)lb * BT + threadIdx.x; n <= Q.y; n += (uint64_t)nlb * BT)
        terms += pc_s1_item(T, Q, pcc, n, &acc);
    acc = pc_block_sum128<BT>(acc, scr);
    terms = pc_block_sum<BT>(terms, scr64);
    if (threadIdx.x == 0) {
        pc_atomic_add128(&Q.sums->s1, acc);
        atomicAdd(&Q.sums->n_s1, terms);
    }
}

__global__ __launch_bounds__(BT) void k_leaf_setup_b(pc_tables T, const pc_query *Qs, pc_blk B)
{
    __shared__ uint64_t scr[BT / 64];
    uint32_t q, lb, nlb;
    pc_blk_of(B, &q, &lb, &nlb);
    const pc_query &Q = Qs[q];
    uint64_t triv = 0, cross = 0;
    for (uint32_t b = lb * BT + threadIdx.x; b <= max(Q.a, Q.c + Q.nb); b += nlb * BT) {
        uint64_t t, c;
        pc_leaf_setup_item(T, Q, b, &t, &c);
        triv += t;
        cross += c;
    }
    const uint64_t s = pc_block_sum<BT>(triv, scr);
    const uint64_t cs = pc_block_sum<BT>(cross, scr);
    if (threadIdx.x == 0) {
        pc_atomic_add128(&Q.sums->s2t, (pc_s128)s);
        atomicAdd(&Q.sums->n_trivial, (unsigned long long)s);
        atomicAdd(&Q.sums->crossings, (unsigned long long)cs);
    }
}

// Exclusive prefix of the counts cnt[0..n) (mode bit stripped) into off
// (which may be cnt itself), the total into *total; the calling workgroup does
// one query in chunks of BT.
__device__ __forceinline__ void pc_escan(const pc_query &Q, const uint64_t *cnt, uint64_t *off,
                                         uint32_t n, uint64_t *total, uint64_t *scr)
{
    uint64_t run = 0;
    for (uint32_t i0 = 0; i0 < n; i0 += BT) {
        const uint32_t i = i0 + threadIdx.x;
        const uint64_t v = i < n ? cnt[i] & ~PC_MODEBIT : 0;
        uint64_t tot;
        const uint64_t ex = pc_block_excl_scan<BT>(v, scr, &tot);
        if (i < n)
            off[i] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0)
        *total = run;
}

// The easy leaves' offsets (candidates: e_off, e_total[0]) and bands
// (singles and groups: e_bk, e_boff, e_total[1], e_total[2]), one workgroup
// per query; then the suffix maxima of the hard-leaf u ranges (pc_ub_suffix).
__global__ __launch_bounds__(BT) void k_escan_b(pc_tables T, const pc_query *Qs)
{
    __shared__ uint64_t scr[BT / 64];
    __shared__ uint64_t sh[BT];
    const pc_query &Q = Qs[blockIdx.x];
    pc_escan(Q, Q.e_count, Q.e_off, Q.a + 1, Q.e_total, scr);
    const uint32_t nband = Q.a / PC_EZ_BAND + 1;
    for (uint32_t g = threadIdx.x; g < nband; g += BT)
        pc_easy_band_item(T, Q, g);
    __syncthreads();
    pc_escan(Q, Q.e_boff, Q.e_boff, nband, Q.e_total + 1, scr);
    pc_escan(Q, Q.e_boff + nband, Q.e_boff + nband, nband, Q.e_total + 2, scr);
    pc_ub_suffix<BT>(Q, sh);
}

__global__ __launch_bounds__(BT) void k_easy_b(pc_tables T, const pc_query *Qs, pc_blk B)
{
    __shared__ pc_s128 scr[BT / 64];
    __shared__ unsigned long long scr64[BT / 64];
    __shared__ uint32_t s_b0, s_g[2];
    uint32_t q, lb, nlb;
    pc_blk_of(B, &q, &lb, &nlb);
    const pc_query &Q = Qs[q];
    unsigned long long nleaf = 0;
    int64_t acc = 0;
    pc_easy_tiles<BT, BEZ_PER>(T, Q, lb, nlb, &s_b0, &acc, &nleaf);
    pc_easy_bands<BT, false>(T, Q, lb, nlb, &s_g[0], &acc);
    pc_easy_bands<BT, true>(T, Q, lb, nlb, &s_g[1], &acc);
    const pc_s128 s = pc_block_sum128<BT>((pc_s128)acc, scr);
    nleaf = pc_block_sum<BT>(nleaf, scr64);
    if (threadIdx.x == 0) {
        pc_atomic_add128(&Q.sums->s2e, s);
        atomicAdd(&Q.sums->n_easy, nleaf);
    }
}

// Carries of whole queries (every row of a query in one pass): block i scans
// the columns [256 cb, 256 cb + 256) of query q down the rows that store them
// (a prefix of the rows: row lengths never grow), carry = sum of the counts
// above, and adds sum w * carry to the query.
__global__ __launch_bounds__(BT) void k_scan_rows_b(const pc_query *Qs, pc_blk B)
{
    __shared__ pc_s128 scr[BT / 64];
    uint32_t q, cb, ncb;
    pc_blk_of(B, &q, &cb, &ncb);
    const pc_query &Q = Qs[q];
    const uint32_t col = cb * BT + threadIdx.x;
    pc_s128 dh = 0, dp = 0;
    const uint64_t nrows = Q.nseg, nb = Q.nb;
    uint64_t carry = 0;
    if (col < nb) { // a sieving column: row r holds it at row_off[r] + col
        for (uint64_t r = 0; r < nrows; r++) {
            const uint64_t o = Q.row_off[r];
            if (col >= Q.row_off[r + 1] - o)
                break;
            const int32_t w = Q.wgt[o + col];
            if (w)
                dh += (pc_s128)w * (pc_s128)carry;
            carry += Q.cnt[o + col];
        }
    } else if (col == nb) { // the P2 column
        for (uint64_t r = 0; r < nrows; r++) {
            const int32_t w = Q.wP[r];
            if (w)
                dp += (pc_s128)w * (pc_s128)carry;
            carry += Q.cntP[r];
        }
    }
    dh = pc_block_sum128<BT>(dh, scr);
    dp = pc_block_sum128<BT>(dp, scr);
    if (threadIdx.x == 0) {
        pc_atomic_add128(&Q.sums->hard_dot, dh);
        pc_atomic_add128(&Q.sums->p2_dot, dp);
    }
}

__global__ void k_combine_b(const pc_query *Qs, uint32_t nq, pc_final *out)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq)
        pc_combine_one(*Qs[q].sums, Qs[q], Qs[q].kx, &out[q]);
}

// A round's results into a caller's array: out[pos[q]] = pi of query q, or all
// ones (pi(x) < 2^63 for every x < 2^64, so never a count) when a quotient
// fell outside its segment in the round or the sum left [0, 2^64).
__global__ void k_batch_out(const pc_final *fin, const uint64_t *pos, uint32_t nq,
                            const int32_t *err, uint64_t *out)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq)
        out[pos[q]] = (*err == 0 && fin[q].ok == 1) ? fin[q].pi : ~0ull;
}

// Results known on the host, as (position, value) pairs, into out.
__global__ void k_scatter_u64(const ulonglong2 *kv, uint64_t n, uint64_t *out)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[kv[i].x] = kv[i].y;
}

hipError_t pc_launch_batch_setup(const pc_tables &T, const pc_query *Qs, const uint32_t *bq_xb,
                                 const uint32_t *bf_xb, uint32_t nb_xb, const uint32_t *bq_s1,
                                 const uint32_t *bf_s1, uint32_t nb_s1, uint32_t nq,
                                 hipStream_t s)
{
    k_xb_b<<<nb_xb, BT, 0, s>>>(T, Qs, pc_blk{bq_xb, bf_xb});
    k_s1_b<<<nb_s1, BT, 0, s>>>(T, Qs, pc_blk{bq_s1, bf_s1});
    k_leaf_setup_b<<<nb_xb, BT, 0, s>>>(T, Qs, pc_blk{bq_xb, bf_xb});
    k_escan_b<<<nq, BT, 0, s>>>(T, Qs);
    return hipGetLastError();
}

hipError_t pc_launch_batch_easy(const pc_tables &T, const pc_query *Qs, const uint32_t *bq,
                                const uint32_t *bf, uint32_t nblocks, hipStream_t s)
{
    k_easy_b<<<nblocks, BT, 0, s>>>(T, Qs, pc_blk{bq, bf});
    return hipGetLastError();
}

hipError_t pc_launch_batch_finish(const pc_query *Qs, const uint32_t *bq, const uint32_t *bf,
                                  uint32_t nblocks, uint32_t nq, pc_final *out, hipStream_t s)
{
    k_scan_rows_b<<<nblocks, BT, 0, s>>>(Qs, pc_blk{bq, bf});
    k_combine_b<<<(nq + 63) / 64, 64, 0, s>>>(Qs, nq, out);
    return hipGetLastError();
}

hipError_t pc_launch_batch_out(const pc_final *fin, const uint64_t *pos, uint32_t nq,
                               const int32_t *err, uint64_t *out, hipStream_t s)
{
    if (nq == 0)
        return hipSuccess;
    k_batch_out<<<(nq + 255) / 256, 256, 0, s>>>(fin, pos, nq, err, out);
    return hipGetLastError();
}

hipError_t pc_launch_scatter_u64(const ulonglong2 *kv, uint64_t n, uint64_t *out, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const uint64_t nb = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
    k_scatter_u64<<<(uint32_t)nb, 256, 0, s>>>(kv, n, out);
    return hipGetLastError();
}

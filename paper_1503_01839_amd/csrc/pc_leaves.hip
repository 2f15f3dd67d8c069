// pc_leaves.hip -- the parts of phi(x, a) = S1 + S2 that need no sieve:
//   S1  ordinary leaves  sum_{n <= y, mu(n) != 0, lpf(n) > p_c} mu(n) phi(x/n, c),
//       phi(u, c) from the wheel (Section 4: phi(m, c) in O(1));
//   S2t trivial special leaves (u = x/(m p_b) < p_b, phi = 1; m is then prime);
//   S2e easy special leaves (p_b <= u < p_b^2, u <= y), Legendre's formula
//       phi(u, b-1) = pi(u) - b + 2 (Section 4), embarrassingly parallel
//       (Section 3);
// and the final combination pi(x) = phi(x, a) + a - 1 - P2.
#include "pc_block.h"
#include "pc_internal.h"

#define LV_T 256
#define PC_MODEBIT (1ull << 63)

// ---------------------------------------------------------------------------
// S1: one lane per n <= y (grid-stride).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LV_T) void k_s1(pc_tables T, pc_query Q, pc_s128 *part)
{
    __shared__ pc_s128 scr[LV_T / 64];
    const uint32_t pc_ = T.primes[Q.c];
    __shared__ unsigned long long scr64[LV_T / 64];
    pc_s128 acc = 0;
    unsigned long long terms = 0;
    const uint64_t stride = (uint64_t)gridDim.x * LV_T;
    for (uint64_t n = 1 + (uint64_t)blockIdx.x * LV_T + threadIdx.x; n <= Q.y; n += stride) {
        const int32_t v = T.mulpf[n];
        const uint32_t l = v < 0 ? (uint32_t)(-v) : (uint32_t)v;
        if (v == 0 || l <= pc_) // mu(n) = 0, or n has a prime factor <= p_c
            continue;
        const uint64_t u = pc_div_any(Q.x, (uint32_t)n);
        const uint64_t qq = pc_div(u, Q.Qc, Q.recip_Qc);
        const uint64_t phi = qq * T.phiQ + T.phitab[u - qq * Q.Qc];
        acc += v > 0 ? (pc_s128)phi : -(pc_s128)phi;
        terms++;
    }
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

// ---------------------------------------------------------------------------
// Per-b setup of the special leaves outside the sieve, c < b < a:
//   trivial leaves: primes m with max(p_b, x/p_b^2) < m <= y  (counted);
//   easy range:     max(y/p_b, H_b, p_b) < m <= min(y, x/p_b^2),
//                   H_b = max(x/p_b^3, x/(p_b (y+1)));
// for p_b^2 > y every m in the range is prime, so the range is stored as
// prime indices; otherwise as candidate m (bit 63 of the count).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LV_T) void k_leaf_setup(pc_tables T, pc_query Q, uint64_t *e_start,
                                                     uint64_t *e_count, pc_s128 *part_t,
                                                     uint64_t *ntriv, ulonglong2 *Ub)
{
    __shared__ uint64_t scr[LV_T / 64];
    const uint32_t b = blockIdx.x * LV_T + threadIdx.x;
    uint64_t triv = 0, cross = 0;
    if (b > Q.c && b <= Q.c + Q.nb) { // a sieving prime
        const uint64_t p = T.primes[b], rp = T.recip[b], X = Q.Xb[b];
        // odd multiples k p_b, k odd, below the sieve end
        cross = (pc_div(Q.sieve_end - 1, p, rp) + 1) / 2;
        // u range of the hard leaves of b: y/p < m <= y, m > p, m <= max(x/p^3, x/(p(y+1)))
        uint64_t m1 = pc_div(Q.y, p, rp) + 1;
        if (m1 < p + 1)
            m1 = p + 1;
        const uint64_t h1 = pc_div(pc_div(X, p, rp), p, rp);
        const uint64_t h2 = pc_div(X, Q.y1, Q.recip_y1);
        uint64_t m2 = h1 > h2 ? h1 : h2;
        if (m2 > Q.y)
            m2 = Q.y;
        ulonglong2 ub;
        ub.x = 1;
        ub.y = 0;
        if (m1 <= m2) {
            ub.x = pc_div_small_q(X, (uint32_t)m2);
            ub.y = pc_div_small_q(X, (uint32_t)m1);
        }
        Ub[b] = ub;
    }
    if (b <= Q.a) {
        uint64_t st = 0, cn = 0;
        if (b > Q.c && b < Q.a) {
            const uint64_t p = T.primes[b], rp = T.recip[b];
            const uint64_t X = Q.Xb[b];
            const uint64_t tp = pc_div(X, p, rp); // floor(x / p^2): u >= p  <=>  m <= tp
            uint64_t m1 = pc_div(Q.y, p, rp) + 1;
            if (m1 < p + 1)
                m1 = p + 1;
            const uint64_t h1 = pc_div(tp, p, rp);
            const uint64_t h2 = pc_div(X, Q.y1, Q.recip_y1);
            const uint64_t H = h1 > h2 ? h1 : h2;
            uint64_t e1 = H + 1 > m1 ? H + 1 : m1;
            uint64_t e2 = tp < Q.y ? tp : Q.y;
            if (p > Q.sqrty) {
                if (e1 <= e2) {
                    const uint64_t k1 = pc_pi_lookup(T.pitab, e1 - 1) + 1;
                    const uint64_t k2 = pc_pi_lookup(T.pitab, e2);
                    if (k1 <= k2) {
                        st = k1;
                        cn = k2 - k1 + 1;
                    }
                }
                // trivial: m prime, m > max(m1 - 1, tp), m <= y
                uint64_t t0 = tp > m1 - 1 ? tp : m1 - 1;
                if (t0 < Q.y)
                    triv = Q.a - pc_pi_lookup(T.pitab, t0);
            } else if (e1 <= e2) {
                st = e1;
                cn = (e2 - e1 + 1) | PC_MODEBIT;
            }
        }
        e_start[b] = st;
        e_count[b] = cn;
    }
    const uint64_t s = pc_block_sum<LV_T>(triv, scr);
    const uint64_t cs = pc_block_sum<LV_T>(cross, scr);
    if (threadIdx.x == 0) {
        part_t[blockIdx.x] = (pc_s128)s;
        atomicAdd((unsigned long long *)ntriv, (unsigned long long)s);
        atomicAdd(&Q.sums->crossings, (unsigned long long)cs);
    }
}

hipError_t pc_launch_leaf_setup(const pc_tables &T, const pc_query &Q, uint64_t *e_start,
                                uint64_t *e_count, pc_s128 *part_trivial, uint64_t *ntrivial,
                                ulonglong2 *Ub, uint32_t nblocks, hipStream_t s)
{
    k_leaf_setup<<<nblocks, LV_T, 0, s>>>(T, Q, e_start, e_count, part_trivial, ntrivial, Ub);
    return hipGetLastError();
}

// e_off[b] = exclusive prefix of the item counts (mode bit stripped)
__global__ void k_strip_counts(const uint64_t *e_count, uint64_t *e_off, uint64_t n)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        e_off[i] = e_count[i] & ~PC_MODEBIT;
}

// ---------------------------------------------------------------------------
// Easy leaves: items laid end to end over b (e_off = exclusive prefix).  A
// workgroup takes tiles of EZ_TILE consecutive items; one search finds the b
// of the tile's first item, then lane t takes items i0 + t, i0 + t + EZ_T, ...
// so neighbouring lanes read neighbouring primes m and neighbouring pi(u)
// entries.  u = x/(m p_b) <= y < 2^50, so the fp64-estimate quotient is exact
// after its remainder check.
// ---------------------------------------------------------------------------
#define EZ_T 256
#define EZ_PER 32
#define EZ_TILE (EZ_T * EZ_PER)

__global__ __launch_bounds__(EZ_T) void k_easy(pc_tables T, pc_query Q, const uint64_t *e_start,
                                               const uint64_t *e_count, const uint64_t *e_off,
                                               const uint64_t *e_total, pc_s128 *part)
{
    __shared__ pc_s128 scr[EZ_T / 64];
    __shared__ unsigned long long scr64[EZ_T / 64];
    __shared__ uint32_t s_b0;
    unsigned long long nleaf = 0;
    const uint64_t E = *e_total;
    int64_t acc = 0;
    for (uint64_t i0 = (uint64_t)blockIdx.x * EZ_TILE; i0 < E; i0 += (uint64_t)gridDim.x * EZ_TILE) {
        if (threadIdx.x == 0) { // b with e_off[b] <= i0 < e_off[b+1], b in [c+1, a-1]
            uint32_t lo_b = Q.c + 1, hi_b = Q.a - 1;
            while (lo_b < hi_b) {
                const uint32_t mid = (lo_b + hi_b + 1) >> 1;
                if (e_off[mid] <= i0)
                    lo_b = mid;
                else
                    hi_b = mid - 1;
            }
            s_b0 = lo_b;
        }
        __syncthreads();
        uint32_t b = s_b0;
        uint64_t off = e_off[b], cn = e_count[b], st = e_start[b], X = Q.Xb[b];
        uint32_t p = T.primes[b];
        const uint64_t iend = i0 + EZ_TILE < E ? i0 + EZ_TILE : E;
        for (uint64_t i = i0 + threadIdx.x; i < iend; i += EZ_T) {
            while (i >= off + (cn & ~PC_MODEBIT)) {
                b++;
                off = e_off[b];
                cn = e_count[b];
                st = e_start[b];
                X = Q.Xb[b];
                p = T.primes[b];
            }
            const uint64_t o = i - off;
            uint32_t m;
            int32_t w;
            if (cn & PC_MODEBIT) {
                m = (uint32_t)(st + o);
                const int32_t v = T.mulpf[m];
                const uint32_t l = v < 0 ? (uint32_t)(-v) : (uint32_t)v;
                if (l <= p) // mu(m) = 0 or lpf(m) <= p_b
                    continue;
                w = v > 0 ? -1 : 1;
            } else {
                m = T.primes[st + o];
                w = 1;
            }
            const uint64_t u = pc_div_small_q(X, m);
            acc += (int64_t)w * ((int64_t)pc_pi_lookup(T.pitab, u) - (int64_t)b + 2);
            nleaf++;
        }
        __syncthreads();
    }
    const pc_s128 s = pc_block_sum128<EZ_T>((pc_s128)acc, scr);
    nleaf = pc_block_sum<EZ_T>(nleaf, scr64);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s;
        atomicAdd(&Q.sums->n_easy, nleaf);
    }
}

hipError_t pc_launch_easy(const pc_tables &T, const pc_query &Q, const uint64_t *e_start,
                          const uint64_t *e_count, const uint64_t *e_off, const uint64_t *e_total,
                          pc_s128 *part, uint32_t nblocks, hipStream_t s)
{
    k_easy<<<nblocks, EZ_T, 0, s>>>(T, Q, e_start, e_count, e_off, e_total, part);
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

// ---------------------------------------------------------------------------
// pi(x) = S1 + S2t + S2e + S2h + a - 1 - P2, with
//   S2h = in-segment sums + sum w * carry, and
//   P2  = sum_{k=a+1}^{kx} (phi(x/p_k, B) + B - 1) - sum_{k=a+1}^{kx} (k - 1),
//   B = c + nb = max(c, bmax) primes crossed by the sieve.
// ---------------------------------------------------------------------------
__global__ void k_combine(const pc_sums *S, pc_query Q, uint64_t kp2, pc_final *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const pc_s128 s2h = S->hard_local + S->hard_dot;
    const pc_s128 B = (pc_s128)(Q.c + Q.nb);
    const pc_s128 a = Q.a, K = kp2;
    pc_s128 p2 = S->p2_local + S->p2_dot;
    if (K > a)
        p2 += (K - a) * (B - 1) - ((K - 1) * K / 2 - (a - 1) * a / 2);
    const pc_s128 phi = S->s1 + S->s2t + S->s2e + s2h;
    const pc_s128 pi = phi + a - 1 - p2;
    out->s1 = S->s1;
    out->s2t = S->s2t;
    out->s2e = S->s2e;
    out->s2h = s2h;
    out->p2 = p2;
    out->phi = phi;
    out->pi = (uint64_t)pi;
    out->ok = (pi >= 0 && (pi >> 64) == 0) ? 1 : 0;
}

hipError_t pc_launch_combine(const pc_sums *sums, const pc_query &Q, uint64_t kp2, pc_final *out,
                             hipStream_t s)
{
    k_combine<<<1, 64, 0, s>>>(sums, Q, kp2, out);
    return hipGetLastError();
}

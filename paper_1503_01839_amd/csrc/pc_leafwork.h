// pc_leafwork.h -- the per-item work of the parts of phi(x, a) = S1 + S2 that
// need no sieve, shared by the one-query kernels (pc_leaves.hip) and the
// batched kernels (pc_batch.hip):
//   S1  ordinary leaves  sum_{n <= y, mu(n) != 0, lpf(n) > p_c} mu(n) phi(x/n, c),
//       phi(u, c) from the wheel (Section 4: phi(m, c) in O(1));
//   S2t trivial special leaves (u = x/(m p_b) < p_b, phi = 1; m is then prime);
//   S2e easy special leaves (p_b <= u < p_b^2, u <= y), Legendre's formula
//       phi(u, b-1) = pi(u) - b + 2 (Section 4), independent of each other
//       (Section 3);
// and the final combination pi(x) = phi(x, a) + a - 1 - P2.
#pragma once

#include "pc_block.h"
#include "pc_internal.h"
#include "pc_leafrange.h"

#define PC_MODEBIT (1ull << 63)

// X_b = floor(x / p_b) for 1 <= b <= a (X_0 = x): its low word, its high
// word (above 2^64, when Xbh is not null) and its value in fp64.
__device__ __forceinline__ void pc_xb_item(const pc_tables &T, const pc_query &Q, uint32_t b)
{
    if (b > Q.a)
        return;
    uint64_t lo, hi = 0;
    if (b == 0) {
        lo = Q.x;
        hi = Q.x_hi;
    } else if (!Q.x_hi) {
        lo = pc_div(Q.x, T.primes[b], T.recip[b]);
    } else {
        lo = pc_div_u128_32(Q.x_hi, Q.x, T.primes[b], &hi, nullptr);
    }
    Q.Xb_w[b] = lo;
    if (Q.Xbh)
        Q.Xbh[b] = (uint32_t)hi;
    Q.Xd[b] = hi ? (double)(((pc_u128)hi << 64) | lo) : (double)lo;
}

// The S1 term of n (pcc = p_c): adds mu(n) phi(x/n, c) to *acc when n <= y is
// squarefree with lpf(n) > p_c, and returns whether it did.
__device__ __forceinline__ bool pc_s1_item(const pc_tables &T, const pc_query &Q, uint32_t pcc,
                                           uint64_t n, pc_s128 *acc)
{
    const int32_t v = T.mulpf[n];
    const uint32_t l = v < 0 ? (uint32_t)(-v) : (uint32_t)v;
    if (v == 0 || l <= pcc) // mu(n) = 0, or n has a prime factor <= p_c
        return false;
    pc_s128 phi;
    if (!Q.x_hi) {
        const uint64_t u = pc_div_any(Q.x, (uint32_t)n);
        const uint64_t qq = pc_div(u, Q.Qc, Q.recip_Qc);
        phi = (pc_s128)(qq * T.phiQ + T.phitab[u - qq * Q.Qc]);
    } else { // above 2^64: u = x / n in 128 bits, u = qq Q_c + r with qq < 2^64
        uint64_t uh;
        const uint64_t ul = pc_div_u128_32(Q.x_hi, Q.x, (uint32_t)n, &uh, nullptr);
        uint32_t r;
        const uint64_t qq = pc_div_wide32(uh, ul, (uint32_t)Q.Qc, &r); // uh < Q_c: x <= 2^72
        phi = (pc_s128)qq * T.phiQ + T.phitab[r];
    }
    *acc += v > 0 ? phi : -phi;
    return true;
}

// Per-b set-up of the special leaves outside the sieve, c < b < a:
//   trivial leaves: primes m with max(p_b, x/p_b^2) < m <= y  (counted);
//   easy range:     max(y/p_b, H_b, p_b) < m <= min(y, x/p_b^2),
//                   H_b = max(x/p_b^3, x/(p_b (y+1)));
// for p_b^2 > y every m in the range is prime, so the range is stored as
// prime indices; otherwise as candidate m (bit 63 of the count).  A prime
// range is cut at s = isqrt(x/p_b): each prime m <= s is a "single"
// (e_start, e_scount); above s, where u = x/(m p_b) < m and consecutive m
// share pi(u), the primes m are taken by the value K = pi(u) instead: those
// with x/(p_b p_{K+1}) < m <= x/(p_b p_K), all with phi(u, b-1) = K - b + 2
// (e_clu; pc_easy_group_term).  For a sieving prime it also records the u
// range of its hard leaves (Ub) and the odd multiples below the sieve end
// (*cross).
__device__ __forceinline__ void pc_leaf_setup_item(const pc_tables &T, const pc_query &Q,
                                                   uint32_t b, uint64_t *triv, uint64_t *cross)
{
    *triv = 0;
    *cross = 0;
    if (b > Q.c && b <= Q.c + Q.nb) { // a sieving prime
        const uint64_t p = T.primes[b], rp = T.recip[b];
        const pc_xv X = pc_xb(Q, b);
        // odd multiples k p_b, k odd, below the sieve end
        *cross = (pc_div(Q.sieve_end - 1, p, rp) + 1) / 2;
        // u range of the hard leaves of b: y/p < m <= y, m > p, m <= max(x/p^3, x/(p(y+1)))
        uint64_t m1 = pc_div(Q.y, p, rp) + 1;
        if (m1 < p + 1)
            m1 = p + 1;
        const uint64_t h1 = pc_div(pc_xv_div(X, (uint32_t)p, rp), p, rp);
        const uint64_t h2 = pc_xv_div64(X, Q.y1, Q.recip_y1);
        uint64_t m2 = h1 > h2 ? h1 : h2;
        if (m2 > Q.y)
            m2 = Q.y;
        ulonglong2 ub;
        ub.x = 1;
        ub.y = 0;
        if (m1 <= m2) {
            ub.x = pc_xv_small_q(X, (uint32_t)m2);
            ub.y = pc_xv_small_q(X, (uint32_t)m1);
        }
        Q.Ub_w[b] = ub;
    }
    if (b <= Q.a) {
        uint64_t st = 0, cn = 0, sn = 0;
        uint4 clu = make_uint4(0, 0, 0, 0);
        if (b > Q.c && b < Q.a) {
            const uint64_t p = T.primes[b], rp = T.recip[b];
            const pc_xv X = pc_xb(Q, b);
            const uint64_t tp = pc_xv_div(X, (uint32_t)p, rp); // floor(x / p^2): u >= p <=> m <= tp
            uint64_t m1 = pc_div(Q.y, p, rp) + 1;
            if (m1 < p + 1)
                m1 = p + 1;
            const uint64_t h1 = pc_div(tp, p, rp);
            const uint64_t h2 = pc_xv_div64(X, Q.y1, Q.recip_y1);
            const uint64_t H = h1 > h2 ? h1 : h2;
            uint64_t e1 = H + 1 > m1 ? H + 1 : m1;
            uint64_t e2 = tp < Q.y ? tp : Q.y;
            if (p > Q.sqrty) {
                if (e1 <= e2) {
                    const uint64_t sx = X.hi ? pc_isqrt_wide(X.hi, X.lo) : pc_isqrt(X.lo);
                    uint64_t s = sx; // single-m items: m <= s
                    if (s < e1 - 1)
                        s = e1 - 1;
                    if (s > e2)
                        s = e2;
                    const uint64_t k1 = pc_pi_lookup(T.pitab, e1 - 1) + 1;
                    const uint64_t ns = pc_pi_lookup(T.pitab, s) + 1 - k1;
                    uint64_t klo = 0, nk = 0;
                    if (s < e2) { // K = pi(u) for u in [X / e2, X / (s + 1)]
                        klo = pc_pi_lookup(T.pitab, pc_xv_small_q(X, (uint32_t)e2));
                        nk = pc_pi_lookup(T.pitab, pc_xv_small_q(X, (uint32_t)(s + 1))) + 1 - klo;
                    }
                    st = k1;
                    sn = ns;
                    clu = make_uint4((uint32_t)nk, (uint32_t)klo, (uint32_t)s, (uint32_t)e2);
                }
                // trivial: m prime, m > max(m1 - 1, tp), m <= y
                uint64_t t0 = tp > m1 - 1 ? tp : m1 - 1;
                if (t0 < Q.y)
                    *triv = Q.a - pc_pi_lookup(T.pitab, t0);
            } else if (e1 <= e2) {
                // every m with lpf(m) > p_b > p_c is prime to p_1..p_c: only
                // those are items, by their wheel numbers (pc_wheel_m)
                st = pc_wheel_count(T, Q, e1 - 1);
                cn = (pc_wheel_count(T, Q, e2) - st) | PC_MODEBIT;
            }
        }
        Q.e_start[b] = st;
        Q.e_count[b] = cn;
        Q.e_scount[b] = sn;
        Q.e_clu[b] = clu;
    }
}

// After the per-b set-up: Ub[b].y becomes the largest u of a hard leaf of any
// sieving prime p_b' with b' >= b, so that in a segment [lo, hi) the columns
// whose Ub.y < lo form a suffix: no prime from there on has a hard leaf at or
// above lo, and the sieve needs neither their counts nor their order (they
// are only cleared).  The calling workgroup (NT threads) does one query.
template <int NT> __device__ __forceinline__ void pc_ub_suffix(const pc_query &Q, uint64_t *sh)
{
    const uint32_t b0 = Q.c + 1, n = Q.nb;
    const uint32_t per = (n + NT - 1) / NT;
    const uint32_t lo = min(n, threadIdx.x * per), hi = min(n, lo + per);
    uint64_t m = 0;
    for (uint32_t i = lo; i < hi; i++)
        m = max(m, Q.Ub_w[b0 + i].y);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (uint32_t d = 1; d < NT; d <<= 1) { // suffix maximum over the threads' pieces
        uint64_t v = sh[threadIdx.x];
        if (threadIdx.x + d < NT)
            v = max(v, sh[threadIdx.x + d]);
        __syncthreads();
        sh[threadIdx.x] = v;
        __syncthreads();
    }
    uint64_t run = threadIdx.x + 1 < NT ? sh[threadIdx.x + 1] : 0;
    for (uint32_t i = hi; i > lo; i--) {
        run = max(run, Q.Ub_w[b0 + i - 1].y);
        Q.Ub_w[b0 + i - 1].y = run;
    }
}

// The group terms of a prime-item b (cl = its e_clu entry: nk, klo, z = s,
// w = e2; bm2 = b - 2).  With C(v) = min(max(v, z), w) and
// V_K = pi(C(X_b / p_K)), the primes m in (max(X_b / p_{K+1}, z),
// min(X_b / p_K, w)] number V_K - V_{K+1} (also when that range is empty, as
// C is monotone), so the part of S2e over K = klo .. khi = klo + nk - 1 is
//   sum_K (V_K - V_{K+1}) (K - bm2)
//     = sum_{klo <= K <= khi + 1} V_K
//       + V_klo (klo - bm2 - 1) - V_{khi+1} (khi + 1 - bm2),
// and its leaves number V_klo - V_{khi+1}.  The sum of the V_K is taken in
// bands (pc_easy_bands), the two end terms once per b (pc_easy_band_item).
// Every quotient is at most y < 2^31 - 1, every p_K < 2^31.
__device__ __forceinline__ int64_t pc_easy_group_v(const pc_tables &T, uint4 cl, uint64_t X,
                                                   double Xd, uint32_t K)
{
    return pc_pi_lookup32(T.pitab,
                          min(max(pc_quot31r(X, Xd, T.primes[K], T.rcpd[K]), cl.z), cl.w));
}

// b in [c+1, a-1] with off[b] <= i0 < off[b+1] (off = an exclusive prefix of
// item counts; the last such b, so b has items).
__device__ __forceinline__ uint32_t pc_item_owner(const pc_query &Q, const uint64_t *off,
                                                  uint64_t i0)
{
    uint32_t lo_b = Q.c + 1, hi_b = Q.a - 1;
    while (lo_b < hi_b) {
        const uint32_t mid = (lo_b + hi_b + 1) >> 1;
        if (off[mid] <= i0)
            lo_b = mid;
        else
            hi_b = mid - 1;
    }
    return lo_b;
}

// The candidate easy leaves (p_b^2 <= y), items (wheel numbers of the m prime
// to p_1..p_c) laid end to end over b (e_off = exclusive prefix of the counts,
// e_total[0] their sum).  The calling
// workgroup (NT threads; every thread calls) takes tiles lb, lb + nlb, ... of
// NT * PER consecutive items; one search finds the b of a tile's first item,
// then thread t takes items i0 + t, i0 + t + NT, ... so neighbouring lanes
// read neighbouring entries.  u = x/(m p_b) <= y < 2^31 - 1, so the
// reciprocal estimate quotient is exact after its remainder check.
template <int NT, int PER>
__device__ __forceinline__ void pc_easy_tiles(const pc_tables &T, const pc_query &Q, uint64_t lb,
                                              uint64_t nlb, uint32_t *s_b0, int64_t *acc,
                                              unsigned long long *nleaf)
{
    constexpr uint64_t TILE = (uint64_t)NT * PER;
    const uint64_t E = Q.e_total[0];
    const uint64_t *e_off = Q.e_off, *e_count = Q.e_count, *e_start = Q.e_start;
    for (uint64_t i0 = lb * TILE; i0 < E; i0 += nlb * TILE) {
        if (threadIdx.x == 0)
            *s_b0 = pc_item_owner(Q, e_off, i0);
        __syncthreads();
        uint32_t b = *s_b0;
        const uint32_t n = (uint32_t)(i0 + TILE < E ? TILE : E - i0); // items of the tile
        uint64_t off = e_off[b], cn = e_count[b] & ~PC_MODEBIT, st = e_start[b], X = Q.Xb[b];
        double Xd = Q.Xd[b];
        uint32_t p = T.primes[b];
        const uint64_t iend = i0 + n;
        for (uint64_t i = i0 + threadIdx.x; i < iend; i += NT) {
            while (i >= off + cn) {
                b++;
                off = e_off[b];
                cn = e_count[b] & ~PC_MODEBIT;
                st = e_start[b];
                X = Q.Xb[b];
                Xd = Q.Xd[b];
                p = T.primes[b];
            }
            const uint32_t m = pc_wheel_m(T, (uint32_t)(st + (i - off)));
            const int32_t v = T.mulpf[m];
            const uint32_t l = v < 0 ? (uint32_t)(-v) : (uint32_t)v;
            if (l <= p) // mu(m) = 0 or lpf(m) <= p_b
                continue;
            const uint32_t u = pc_quot31(X, Xd, m); // u <= y < 2^31 - 1
            const int64_t phi = (int64_t)pc_pi_lookup32(T.pitab, u) - (int64_t)b + 2;
            *acc += v > 0 ? -phi : phi; // -mu(m) phi(u, b-1)
            (*nleaf)++;
        }
        __syncthreads();
    }
}

// The bands of the singles and groups (layout in pc_query): for band g, the
// first and one past the last prime index of each kind over the band's b, and
// its units; and the parts of S2e and of the
// leaf count that the bands' sums leave out: -(b - 2) for each single
// (pc_easy_bands adds pi(u) alone), the two end terms of each b's groups
// (pc_easy_group_v), and every single and group leaf.
__device__ __forceinline__ void pc_easy_band_item(const pc_tables &T, const pc_query &Q,
                                                  uint32_t g)
{
    const uint32_t nband = Q.a / PC_EZ_BAND + 1;
    if (g >= nband)
        return;
    const uint32_t b0 = g * PC_EZ_BAND, b1 = min(b0 + PC_EZ_BAND, Q.a + 1);
    uint32_t s_lo = UINT32_MAX, s_hi = 0, g_lo = UINT32_MAX, g_hi = 0;
    pc_s128 cst = 0;
    int64_t leaves = 0;
    unsigned long long terms = 0;
    for (uint32_t b = b0; b < b1; b++) {
        const uint64_t X = Q.Xb[b];
        const double Xd = Q.Xd[b];
        const uint32_t ns = (uint32_t)Q.e_scount[b];
        if (ns) {
            const uint32_t k1 = (uint32_t)Q.e_start[b];
            s_lo = min(s_lo, k1);
            s_hi = max(s_hi, k1 + ns);
            cst -= (pc_s128)ns * (b - 2);
            leaves += ns;
            terms += ns;
        }
        const uint4 cl = Q.e_clu[b];
        if (cl.x) {
            const uint32_t klo = cl.y, khi1 = cl.y + cl.x; // K = klo .. khi1
            g_lo = min(g_lo, klo);
            g_hi = max(g_hi, khi1 + 1);
            const int64_t v0 = pc_easy_group_v(T, cl, X, Xd, klo);
            const int64_t v1 = pc_easy_group_v(T, cl, X, Xd, khi1);
            cst += (pc_s128)v0 * (int64_t)(klo - b + 1) - (pc_s128)v1 * (int64_t)(khi1 + 2 - b);
            leaves += v0 - v1;
            terms += cl.x + 1;
        }
    }
    if (cst != 0)
        pc_atomic_add128(&Q.sums->s2e, cst);
    if (leaves)
        atomicAdd(&Q.sums->n_easy, (unsigned long long)leaves);
    if (terms)
        atomicAdd(&Q.sums->n_easy_terms, terms);
    Q.e_bk[g] = s_lo;
    Q.e_boff[g] = s_hi > s_lo ? (s_hi - s_lo + PC_EZ_UNIT - 1) / PC_EZ_UNIT : 0;
    Q.e_bk[nband + g] = g_lo;
    Q.e_boff[nband + g] = g_hi > g_lo ? (g_hi - g_lo + PC_EZ_UNIT - 1) / PC_EZ_UNIT : 0;
}

// Singles (GRP false) or groups (GRP true) of the easy leaves, in units of
// PC_EZ_UNIT prime indices k (one per thread; NT = PC_EZ_UNIT) against the
// PC_EZ_BAND b of a band (layout in pc_query).  The calling workgroup takes the
// contiguous units [U lb / nlb, U (lb + 1) / nlb).  A thread loads p_k and 1/p_k
// once per unit; for each b of the band that has k in its range it adds
//   singles: pi(u), u = X_b / p_k;
//   groups:  V_k = pi(C(X_b / p_k)) (pc_easy_group_v);
// the rest of each term is added once per b (pc_easy_band_item).  Every
// thread takes every b (a lane outside the b's range looks up pi(2) and drops
// it), so the loop has no branches; band data are uniform over the workgroup.
template <int NT, bool GRP>
__device__ __forceinline__ void pc_easy_bands(const pc_tables &T, const pc_query &Q, uint64_t lb,
                                              uint64_t nlb, uint32_t *s_g, int64_t *acc)
{
    static_assert(NT == PC_EZ_UNIT, "one thread per prime index of a unit");
    const uint32_t nband = Q.a / PC_EZ_BAND + 1;
    const uint64_t *boff = Q.e_boff + (GRP ? nband : 0);
    const uint32_t *bk = Q.e_bk + (GRP ? nband : 0);
    const uint64_t U = Q.e_total[GRP ? 2 : 1];
    const uint64_t u0 = U * lb / nlb, u1 = U * (lb + 1) / nlb;
    if (u0 >= u1)
        return;
    if (threadIdx.x == 0) { // the band of unit u0: last g with boff[g] <= u0
        uint32_t lo = 0, hi = nband - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (boff[mid] <= u0)
                lo = mid;
            else
                hi = mid - 1;
        }
        *s_g = lo;
    }
    __syncthreads();
    uint32_t g = __builtin_amdgcn_readfirstlane(*s_g);
    uint64_t gend = g + 1 < nband ? boff[g + 1] : U;
    int64_t a = 0;
    const uint32_t kcap = Q.a + 1; // p_k and 1/p_k exist for k <= a + 1
    for (uint64_t u = u0; u < u1; u++) {
        while (u >= gend) {
            g++;
            gend = g + 1 < nband ? boff[g + 1] : U;
        }
        const uint32_t k = bk[g] + (uint32_t)(u - boff[g]) * PC_EZ_UNIT + threadIdx.x;
        const uint32_t kk = min(k, kcap);
        const uint32_t m = T.primes[kk];
        const double rm = T.rcpd[kk];
        const uint32_t b1 = min(g * PC_EZ_BAND + PC_EZ_BAND, Q.a + 1);
#pragma unroll 4
        for (uint32_t b = g * PC_EZ_BAND; b < b1; b++) {
            bool in;
            uint32_t q = pc_quot31r(Q.Xb[b], Q.Xd[b], m, rm);
            if constexpr (!GRP) {
                in = k - (uint32_t)Q.e_start[b] < (uint32_t)Q.e_scount[b];
            } else {
                const uint4 cl = Q.e_clu[b];
                in = (k - cl.y <= cl.x) && cl.x != 0;
                q = min(max(q, cl.z), cl.w);
            }
            const uint32_t v = pc_pi_lookup32(T.pitab, in ? q : 2u);
            a += in ? v : 0u;
        }
    }
    *acc += a;
}

// pi(x) = S1 + S2t + S2e + S2h + a - 1 - P2, with
//   S2h = in-segment sums + sum w * carry, and
//   P2  = sum_{k=a+1}^{kx} (phi(x/p_k, B) + B - 1) - sum_{k=a+1}^{kx} (k - 1),
//   B = c + nb = max(c, bmax) primes crossed by the sieve.
__device__ __forceinline__ void pc_combine_one(const pc_sums &S, const pc_query &Q, uint64_t kp2,
                                               pc_final *out)
{
    const pc_s128 s2h = S.hard_local + S.hard_dot;
    const pc_s128 B = (pc_s128)(Q.c + Q.nb);
    const pc_s128 a = Q.a, K = kp2;
    pc_s128 p2 = S.p2_local + S.p2_dot;
    if (K > a)
        p2 += (K - a) * (B - 1) - ((K - 1) * K / 2 - (a - 1) * a / 2);
    const pc_s128 phi = S.s1 + S.s2t + S.s2e + s2h;
    const pc_s128 pi = phi + a - 1 - p2;
    out->s1 = S.s1;
    out->s2t = S.s2t;
    out->s2e = S.s2e;
    out->s2h = s2h;
    out->p2 = p2;
    out->phi = phi;
    out->pi = (uint64_t)pi;
    out->pi_hi = (uint64_t)(pi >> 64);
    out->ok = pi < 0 ? 0 : (pi >> 64) == 0 ? 1 : 2;
}

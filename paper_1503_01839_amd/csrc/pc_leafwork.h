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

#define PC_MODEBIT (1ull << 63)

// X_b = floor(x / p_b) for 1 <= b <= a (X_0 = x).
__device__ __forceinline__ void pc_xb_item(const pc_tables &T, const pc_query &Q, uint32_t b)
{
    if (b == 0)
        Q.Xb_w[0] = Q.x;
    else if (b <= Q.a)
        Q.Xb_w[b] = pc_div(Q.x, T.primes[b], T.recip[b]);
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
    const uint64_t u = pc_div_any(Q.x, (uint32_t)n);
    const uint64_t qq = pc_div(u, Q.Qc, Q.recip_Qc);
    const uint64_t phi = qq * T.phiQ + T.phitab[u - qq * Q.Qc];
    *acc += v > 0 ? (pc_s128)phi : -(pc_s128)phi;
    return true;
}

// Per-b set-up of the special leaves outside the sieve, c < b < a:
//   trivial leaves: primes m with max(p_b, x/p_b^2) < m <= y  (counted);
//   easy range:     max(y/p_b, H_b, p_b) < m <= min(y, x/p_b^2),
//                   H_b = max(x/p_b^3, x/(p_b (y+1)));
// for p_b^2 > y every m in the range is prime, so the range is stored as
// prime indices; otherwise as candidate m (bit 63 of the count).  A prime
// range is cut at s = 1.5 isqrt(x/p_b): each m <= s is one item; above s,
// where u = x/(m p_b) < m and consecutive m share pi(u), the items are the
// values K = pi(u) instead, each standing for the primes m with
// x/(p_b p_{K+1}) < m <= x/(p_b p_K), all with phi(u, b-1) = K - b + 2.  For a
// sieving prime it also records the u range of its hard leaves (Ub) and the
// odd multiples below the sieve end (*cross).
__device__ __forceinline__ void pc_leaf_setup_item(const pc_tables &T, const pc_query &Q,
                                                   uint32_t b, uint64_t *triv, uint64_t *cross)
{
    *triv = 0;
    *cross = 0;
    if (b > Q.c && b <= Q.c + Q.nb) { // a sieving prime
        const uint64_t p = T.primes[b], rp = T.recip[b], X = Q.Xb[b];
        // odd multiples k p_b, k odd, below the sieve end
        *cross = (pc_div(Q.sieve_end - 1, p, rp) + 1) / 2;
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
        Q.Ub_w[b] = ub;
    }
    if (b <= Q.a) {
        uint64_t st = 0, cn = 0;
        uint4 clu = make_uint4(0, 0, 0, 0);
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
                    const uint64_t sx = pc_isqrt(X);
                    uint64_t s = sx + sx / 2; // single-m items: m <= s
                    if (s < e1 - 1)
                        s = e1 - 1;
                    if (s > e2)
                        s = e2;
                    const uint64_t k1 = pc_pi_lookup(T.pitab, e1 - 1) + 1;
                    const uint64_t ns = pc_pi_lookup(T.pitab, s) + 1 - k1;
                    uint64_t klo = 0, nk = 0;
                    if (s < e2) { // K = pi(u) for u in [X / e2, X / (s + 1)]
                        klo = pc_pi_lookup(T.pitab, pc_div_any(X, (uint32_t)e2));
                        nk = pc_pi_lookup(T.pitab, pc_div_any(X, (uint32_t)(s + 1))) + 1 - klo;
                    }
                    if (ns + nk) {
                        st = k1;
                        cn = ns + nk;
                        clu = make_uint4((uint32_t)ns, (uint32_t)klo, (uint32_t)s, (uint32_t)e2);
                    }
                }
                // trivial: m prime, m > max(m1 - 1, tp), m <= y
                uint64_t t0 = tp > m1 - 1 ? tp : m1 - 1;
                if (t0 < Q.y)
                    *triv = Q.a - pc_pi_lookup(T.pitab, t0);
            } else if (e1 <= e2) {
                st = e1;
                cn = (e2 - e1 + 1) | PC_MODEBIT;
            }
        }
        Q.e_start[b] = st;
        Q.e_count[b] = cn;
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

// Item o of a prime-item b (cl = its e_clu entry, st its first prime index,
// bm2 = b - 2, Xd = (double)X_b): the prime m = p_{st+o} for o < cl.x, else
// K = cl.y + o - cl.x and the primes m in (max(X_b / p_{K+1}, cl.z),
// min(X_b / p_K, cl.w)].  Adds the item's part of S2e to *acc and its
// leaves to *nl.  Every quotient is at most y < 2^32 - 1.
__device__ __forceinline__ void pc_easy_prime_item(const pc_tables &T, uint4 cl, uint32_t st,
                                                   uint64_t X, double Xd, uint32_t bm2, uint32_t o,
                                                   int64_t *acc, uint32_t *nl)
{
    if (o < cl.x) {
        const uint32_t u = pc_quot32(X, Xd, T.primes[st + o]); // p_b <= u <= y
        *acc += pc_pi_lookup32(T.pitab, u) - bm2;              // phi(u, b-1) = pi(u) - b + 2
        (*nl)++;
    } else {
        const uint32_t K = cl.y + (o - cl.x);
        const uint32_t hi = min(pc_quot32(X, Xd, T.primes[K]), cl.w);
        const uint32_t lo = max(pc_quot32(X, Xd, T.primes[K + 1]), cl.z);
        if (hi > lo) {
            const uint32_t n = pc_pi_lookup32(T.pitab, hi) - pc_pi_lookup32(T.pitab, lo);
            *acc += (int64_t)n * (int64_t)(K - bm2);
            *nl += n;
        }
    }
}

// Easy leaves, items laid end to end over b (e_off = exclusive prefix of the
// counts, e_total their sum).  The calling workgroup (NT threads; every thread
// calls) takes tiles lb, lb + nlb, ... of NT * PER consecutive items; one
// search finds the b of a tile's first item, then thread t takes items
// i0 + t, i0 + t + NT, ... so neighbouring lanes read neighbouring primes m
// and neighbouring pi(u) entries.  u = x/(m p_b) <= y < 2^32 - 1, so the
// reciprocal estimate quotient is exact after its remainder check.  The
// candidate-m items (p_b^2 <= y) all precede the prime items (p_b^2 > y), so a
// tile that starts in a prime range has only prime items (single primes m,
// -mu(m) = 1, or groups of them sharing K = pi(u); pc_easy_prime_item), and
// its loop needs no filter.
template <int NT, int PER>
__device__ __forceinline__ void pc_easy_tiles(const pc_tables &T, const pc_query &Q, uint64_t lb,
                                              uint64_t nlb, uint32_t *s_b0, int64_t *acc,
                                              unsigned long long *nleaf)
{
    constexpr uint64_t TILE = (uint64_t)NT * PER;
    const uint64_t E = *Q.e_total;
    const uint64_t *e_off = Q.e_off, *e_count = Q.e_count, *e_start = Q.e_start;
    for (uint64_t i0 = lb * TILE; i0 < E; i0 += nlb * TILE) {
        if (threadIdx.x == 0) { // b with e_off[b] <= i0 < e_off[b+1], b in [c+1, a-1]
            uint32_t lo_b = Q.c + 1, hi_b = Q.a - 1;
            while (lo_b < hi_b) {
                const uint32_t mid = (lo_b + hi_b + 1) >> 1;
                if (e_off[mid] <= i0)
                    lo_b = mid;
                else
                    hi_b = mid - 1;
            }
            *s_b0 = lo_b;
        }
        __syncthreads();
        uint32_t b = *s_b0;
        const uint32_t n = (uint32_t)(i0 + TILE < E ? TILE : E - i0); // items of the tile
        uint64_t cn = e_count[b];
        if (!(cn & PC_MODEBIT)) {
            // prime items only; item t of the tile is item t - rs of its b
            int64_t rs = (int64_t)(e_off[b] - i0), re = rs + (int64_t)cn;
            uint32_t st = (uint32_t)e_start[b], bm2 = b - 2;
            uint4 cl = Q.e_clu[b];
            uint64_t X = Q.Xb[b];
            double Xd = (double)X;
            int64_t a = 0;
            uint32_t nl = 0;
            for (uint32_t t = threadIdx.x; t < n; t += NT) {
                while ((int64_t)t >= re) {
                    b++;
                    rs = re;
                    re = rs + (int64_t)e_count[b];
                    st = (uint32_t)e_start[b];
                    cl = Q.e_clu[b];
                    bm2 = b - 2;
                    X = Q.Xb[b];
                    Xd = (double)X;
                }
                pc_easy_prime_item(T, cl, st, X, Xd, bm2, (uint32_t)((int64_t)t - rs), &a, &nl);
            }
            *acc += a;
            *nleaf += nl;
        } else {
            uint64_t off = e_off[b], st = e_start[b], X = Q.Xb[b];
            double Xd = (double)X;
            uint32_t p = T.primes[b];
            const uint64_t iend = i0 + n;
            for (uint64_t i = i0 + threadIdx.x; i < iend; i += NT) {
                while (i >= off + (cn & ~PC_MODEBIT)) {
                    b++;
                    off = e_off[b];
                    cn = e_count[b];
                    st = e_start[b];
                    X = Q.Xb[b];
                    Xd = (double)X;
                    p = T.primes[b];
                }
                const uint64_t o = i - off;
                if (!(cn & PC_MODEBIT)) { // a prime-item b past the tile's start
                    int64_t a = 0;
                    uint32_t nl = 0;
                    pc_easy_prime_item(T, Q.e_clu[b], (uint32_t)st, X, Xd, b - 2, (uint32_t)o, &a,
                                       &nl);
                    *acc += a;
                    *nleaf += nl;
                    continue;
                }
                const uint32_t m = (uint32_t)(st + o);
                const int32_t v = T.mulpf[m];
                const uint32_t l = v < 0 ? (uint32_t)(-v) : (uint32_t)v;
                if (l <= p) // mu(m) = 0 or lpf(m) <= p_b
                    continue;
                const uint32_t u = pc_quot32(X, Xd, m); // u <= y < 2^32 - 1
                const int64_t phi = (int64_t)pc_pi_lookup32(T.pitab, u) - (int64_t)b + 2;
                *acc += v > 0 ? -phi : phi; // -mu(m) phi(u, b-1)
                (*nleaf)++;
            }
        }
        __syncthreads();
    }
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
    out->ok = (pi >= 0 && (pi >> 64) == 0) ? 1 : 0;
}

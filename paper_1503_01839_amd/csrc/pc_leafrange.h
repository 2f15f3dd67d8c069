// pc_leafrange.h -- the hard special leaves of one sieving prime that land in
// one segment (Sections 2.3 and 3 of the paper): shared by the sieve kernel and
// the tile planner.
#pragma once

#include "pc_device.h"
#include "pc_internal.h"

#define PC_CAND 0x80000000u

// Candidates m for a prime p_b <= sqrt(y) are the integers prime to
// p_1..p_c (lpf(m) > p_b > p_c implies it), numbered from 0 in increasing
// order: candidate k is Q_c (k / phi(Q_c)) + wres[k mod phi(Q_c)], and the
// candidates up to m number phi(m, c) = phi(Q_c) (m / Q_c) + phitab[m mod Q_c].
__device__ __forceinline__ uint32_t pc_wheel_m(const pc_tables &T, uint32_t k)
{
    uint32_t q = (uint32_t)((float)k * T.rphiQ); // within one of k / phi(Q_c) (k < 2^24 phi(Q_c))
    int32_t r = (int32_t)(k - q * T.phiQ);
    if (r < 0) {
        q--;
        r += (int32_t)T.phiQ;
    } else if (r >= (int32_t)T.phiQ) {
        q++;
        r -= (int32_t)T.phiQ;
    }
    return q * T.Qc + T.wres[r];
}

__device__ __forceinline__ uint64_t pc_wheel_count(const pc_tables &T, const pc_query &Q, uint64_t m)
{
    const uint64_t q = pc_div(m, Q.Qc, Q.recip_Qc);
    return q * T.phiQ + T.phitab[m - q * Q.Qc];
}

// The hard leaves (b, m) whose u = floor(X_b/m) lies in [lo, hi): special
// (y/p_b < m <= y, lpf(m) > p_b) and hard (m <= max(x/p^3, x/(p(y+1)))).
// For p_b^2 > y every such m is prime and the range is returned as prime
// indices [ls, ls + lc); otherwise as candidate numbers (pc_wheel_m),
// lc | PC_CAND.
__device__ __forceinline__ void pc_leaf_mrange(const pc_query &Q, uint32_t b, uint64_t p,
                                               uint64_t rp, uint64_t lo, uint64_t hi,
                                               uint64_t rhi, uint64_t rlo, uint64_t *m1o,
                                               uint64_t *m2o)
{
    const pc_xv X = pc_xb(Q, b);
    const uint64_t mA = pc_xv_div64(X, hi, rhi) + 1;                // u < hi   <=> m > X/hi
    const uint64_t mB = lo ? pc_xv_div64(X, lo, rlo) : Q.y;          // u >= lo  <=> m <= X/lo
    uint64_t m1 = pc_div(Q.y, p, rp) + 1;
    if (m1 < mA)
        m1 = mA;
    if (m1 < p + 1)
        m1 = p + 1;
    const uint64_t h1 = pc_div(pc_xv_div(X, (uint32_t)p, rp), p, rp);
    const uint64_t h2 = pc_xv_div64(X, Q.y1, Q.recip_y1);
    uint64_t m2 = h1 > h2 ? h1 : h2;
    if (m2 > Q.y)
        m2 = Q.y;
    if (m2 > mB)
        m2 = mB;
    *m1o = m1;
    *m2o = m2;
}

__device__ __forceinline__ void pc_leaf_range(const pc_tables &TB, const pc_query &Q, uint32_t b,
                                              uint64_t p, uint64_t rp, uint64_t lo, uint64_t hi,
                                              uint64_t rhi, uint64_t rlo, uint32_t *ls,
                                              uint32_t *lc)
{
    uint64_t m1, m2;
    pc_leaf_mrange(Q, b, p, rp, lo, hi, rhi, rlo, &m1, &m2);
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
            const uint64_t k1 = pc_wheel_count(TB, Q, m1 - 1), k2 = pc_wheel_count(TB, Q, m2);
            if (k1 < k2) {
                *ls = (uint32_t)k1;
                *lc = (uint32_t)(k2 - k1) | PC_CAND;
            }
        }
    }
}


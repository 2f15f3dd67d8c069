// pc_device.h -- integer helpers shared by the gfx950 kernels and the host
// planner of the prime-counting library.
//
// All arithmetic of the method is exact integer arithmetic.  The GPU has no
// integer divide instruction, so every quotient on a hot path is formed by a
// multiply-high with a precomputed 64-bit reciprocal of the divisor and one
// correction step (division by invariant integers, Granlund & Montgomery,
// PLDI 1994), or -- for divisors that change per lane -- from an fp64
// estimate corrected by an exact integer remainder test.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned __int128 pc_u128;
typedef __int128 pc_s128;

#define PC_HD __host__ __device__ __forceinline__

// r = floor((2^64 - 1) / d) for d >= 1.
PC_HD uint64_t pc_recip(uint64_t d) { return ~0ull / d; }

PC_HD uint64_t pc_mulhi(uint64_t a, uint64_t b)
{
    return (uint64_t)(((pc_u128)a * b) >> 64);
}

// floor(n / d) given r = pc_recip(d).  For any n < 2^64 and d >= 1:
// n*r/2^64 = n/d - n(1+e)/(d 2^64) with e = (2^64-1) mod d < d, which lies in
// (n/d - 1, n/d]; so q0 = mulhi(n, r) is floor(n/d) or one less.
PC_HD uint64_t pc_div(uint64_t n, uint64_t d, uint64_t r)
{
    uint64_t q = pc_mulhi(n, r);
    uint64_t rem = n - q * d;
    if (rem >= d)
        q++;
    return q;
}

// floor(n / d) for d < 2^32 when the quotient is known to be < 2^50: the
// fp64 estimate has relative error below 2^-51, so it is within 1 of the
// true quotient and one signed remainder test fixes it.
PC_HD uint64_t pc_div_small_q(uint64_t n, uint32_t d)
{
    uint64_t q = (uint64_t)((double)n / (double)d);
    int64_t rem = (int64_t)(n - q * (uint64_t)d);
    if (rem < 0)
        q--;
    else if (rem >= (int64_t)d)
        q++;
    return q;
}

// Quotients on the leaf paths, where the divisor changes from lane to lane
// and the dividend is shared (the caller converts it to fp64 once).  1/d is
// the hardware fp64 reciprocal estimate refined by two Newton steps; each
// step squares the relative error, so any estimate better than 2^-20 ends
// within a few units of 2^-52.  The product with fl(n) is then within
// n/d * 2^-49 of n/d, under 1/4 for n/d < 2^47, and the truncated estimate
// is floor(n/d) or one off, which one exact remainder test corrects.
__device__ __forceinline__ double pc_rcp_f64(uint32_t d)
{
    const double dd = (double)d;
    double r = __builtin_amdgcn_rcp(dd);
    r = __builtin_fma(__builtin_fma(-dd, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-dd, r, 1.0), r, r);
    return r;
}

// floor(n / d) for 1 <= d < 2^32 when the quotient is known to be below
// 2^32 - 1; nd = (double)n.  The estimate is raised by 2^-10, more than its
// error (2^-17 here), so the truncation is floor(n/d) or one above it, and
// only the sign of the remainder needs testing.
__device__ __forceinline__ uint32_t pc_quot32(uint64_t n, double nd, uint32_t d)
{
    const uint32_t q = (uint32_t)__builtin_fma(nd, pc_rcp_f64(d), 0x1p-10);
    const int64_t rem = (int64_t)(n - (uint64_t)q * d);
    return q - (rem < 0 ? 1u : 0u);
}

// pc_quot32 for divisors d < 2^31, with rd = 1/d correctly rounded (a table
// entry): the estimate's error is then below 2^-19, well under the same 2^-10
// margin, and the remainder n - q d of the estimate q lies in [-d, d), so its
// low 32 bits read as a signed number are its value.
__device__ __forceinline__ uint32_t pc_quot31r(uint64_t n, double nd, uint32_t d, double rd)
{
    const uint32_t q = (uint32_t)__builtin_fma(nd, rd, 0x1p-10);
    const int32_t rem = (int32_t)((uint32_t)n - q * d);
    return q - (rem < 0 ? 1u : 0u);
}

// pc_quot31r with 1/d from pc_rcp_f64.
__device__ __forceinline__ uint32_t pc_quot31(uint64_t n, double nd, uint32_t d)
{
    const uint32_t q = (uint32_t)__builtin_fma(nd, pc_rcp_f64(d), 0x1p-10);
    const int32_t rem = (int32_t)((uint32_t)n - q * d);
    return q - (rem < 0 ? 1u : 0u);
}

// pc_quot_in for a 64-bit divisor 2^32 <= d < 2^40 (the primes above 2^32 of
// P2 when x > 2^64): n is x modulo 2^64 and nd the rounded x; the remainder of
// the estimate, formed modulo 2^64, is small and exact.
__device__ __forceinline__ bool pc_quot_in64(uint64_t n, double nd, uint64_t d, uint64_t base,
                                             uint32_t span, uint32_t *off)
{
    const double t = nd / (double)d - (double)base;
    if (!(t > -2.0 && t < (double)span + 2.0))
        return false;
    int32_t q = (int32_t)t;
    const int64_t rem = (int64_t)(n - (base + (uint64_t)(int64_t)q) * d);
    if (rem < 0)
        q--;
    else if (rem >= (int64_t)d)
        q++;
    *off = (uint32_t)q;
    return q >= 0 && (uint32_t)q < span;
}

// floor(n / d) - base for 1 <= d < 2^32, base < 2^47, n/d < 2^47:
// returns false if the quotient lies outside [base, base + span), span <
// 2^30, else true with *off = the quotient - base.  nd = (double)n.
__device__ __forceinline__ bool pc_quot_in(uint64_t n, double nd, uint32_t d, uint64_t base,
                                           uint32_t span, uint32_t *off)
{
    const double t = nd * pc_rcp_f64(d) - (double)base;
    if (!(t > -2.0 && t < (double)span + 2.0))
        return false;
    int32_t q = (int32_t)t;
    const int64_t rem = (int64_t)(n - (base + (uint64_t)(int64_t)q) * d);
    if (rem < 0)
        q--;
    else if (rem >= (int64_t)d)
        q++;
    *off = (uint32_t)q;
    return q >= 0 && (uint32_t)q < span;
}

// Exact floor(n / d) for any n < 2^64, 1 <= d < 2^32: fp64 estimate, one
// exact refinement of the remainder, then a final one-step correction.
PC_HD uint64_t pc_div_any(uint64_t n, uint32_t d)
{
    if (d == 1)
        return n;
    double dd = (double)d;
    uint64_t q = (uint64_t)((double)n / dd);      // q <= 2^63, within 2^11 of the truth
    int64_t rem = (int64_t)(n - q * (uint64_t)d); // |rem| <= 2^11 d < 2^43
    q += (int64_t)((double)rem / dd);             // now within 1
    rem = (int64_t)(n - q * (uint64_t)d);
    while (rem < 0) {
        q--;
        rem += d;
    }
    while (rem >= (int64_t)d) {
        q++;
        rem -= d;
    }
    return q;
}

// Queries above 2^64: x = hi 2^64 + lo (x <= 2^72).
//
// floor((hi 2^64 + lo) / d) for 1 <= d < 2^32 and hi < d (so the quotient is
// below 2^64), by long division in base 2^32; *rem receives the remainder.
PC_HD uint64_t pc_div_wide32(uint64_t hi, uint64_t lo, uint32_t d, uint32_t *rem)
{
    uint64_t r = hi;
    const uint64_t n1 = (r << 32) | (lo >> 32);
    const uint64_t q1 = n1 / d;
    r = n1 - q1 * d;
    const uint64_t n0 = (r << 32) | (lo & 0xFFFFFFFFull);
    const uint64_t q0 = n0 / d;
    if (rem)
        *rem = (uint32_t)(n0 - q0 * d);
    return (q1 << 32) | q0;
}

// floor(x / d) for x = hi 2^64 + lo (xd = x rounded to double) when the
// quotient is below 2^64 and d < 2^46: the fp64 estimate q0 is within
// q 2^-51 + 1 < 2^13 of the quotient, so the remainder x - q0 d, formed
// modulo 2^64, is a signed number below 2^59 in size; one integer division of
// it brings the estimate within one, and the remainder's sign settles it.
PC_HD uint64_t pc_div_wide(uint64_t lo, double xd, uint64_t d)
{
    const double t = xd / (double)d;
    uint64_t q = t < 0x1p64 ? (uint64_t)t : ~0ull;
    int64_t rem = (int64_t)(lo - q * d);
    q += rem / (int64_t)d;
    rem = (int64_t)(lo - q * d);
    while (rem < 0) {
        q--;
        rem += (int64_t)d;
    }
    while (rem >= (int64_t)d) {
        q++;
        rem -= (int64_t)d;
    }
    return q;
}

// floor(x / d) for x = hi 2^64 + lo, 1 <= d < 2^32, any hi: the quotient's
// high word in *qhi, its low word returned (long division in base 2^32).
PC_HD uint64_t pc_div_u128_32(uint64_t hi, uint64_t lo, uint32_t d, uint64_t *qhi, uint32_t *rem)
{
    *qhi = hi / d;
    return pc_div_wide32(hi % d, lo, d, rem);
}

// floor(x / d) for 1 <= d < 2^32 when the quotient is below 2^50, x given as
// its low word lo and its value xd in fp64 (x may exceed 2^64): the estimate
// is within one of the quotient and the remainder, formed modulo 2^64, is
// exact.  For x < 2^64 this is pc_div_small_q.
PC_HD uint64_t pc_div_small_qd(uint64_t lo, double xd, uint32_t d)
{
    uint64_t q = (uint64_t)(xd / (double)d);
    const int64_t rem = (int64_t)(lo - q * (uint64_t)d);
    if (rem < 0)
        q--;
    else if (rem >= (int64_t)d)
        q++;
    return q;
}

// isqrt(hi 2^64 + lo) for values below 2^126: the fp64 root is within one of
// the integer root below 2^104, and the loops settle it.
PC_HD uint64_t pc_isqrt_wide(uint64_t hi, uint64_t lo)
{
    const pc_u128 n = ((pc_u128)hi << 64) | lo;
    uint64_t r = (uint64_t)__builtin_sqrt((double)n);
    while (r > 0 && (pc_u128)r * r > n)
        r--;
    while ((pc_u128)(r + 1) * (r + 1) <= n)
        r++;
    return r;
}

// Integer square and cube roots, exact (used by the host planner).
PC_HD uint64_t pc_isqrt(uint64_t n)
{
    uint64_t r = (uint64_t)__builtin_sqrt((double)n);
    while (r > 0 && (pc_u128)r * r > n)
        r--;
    while ((pc_u128)(r + 1) * (r + 1) <= n)
        r++;
    return r;
}

PC_HD uint64_t pc_icbrt(uint64_t n)
{
    uint64_t r = (uint64_t)__builtin_cbrt((double)n);
    while (r > 0 && (pc_u128)r * r * r > n)
        r--;
    while ((pc_u128)(r + 1) * (r + 1) * (r + 1) <= n)
        r++;
    return r;
}

// pi table: entry e holds a 32-bit mask of the odd numbers 64e+1 .. 64e+63
// (bit j <-> 64e + 2j + 1 is prime) and the number of odd primes below 64e.
// pi(n) = [n >= 2] + (odd primes <= n).
PC_HD uint32_t pc_pi_lookup(const uint2 *tab, uint64_t n)
{
    if (n < 2)
        return 0;
    uint64_t i = (n - 1) >> 1; // odd index of the largest odd number <= n
    uint2 e = tab[i >> 5];
    uint32_t sh = 31u - (uint32_t)(i & 31);
    return 1u + e.y + (uint32_t)__builtin_popcount((e.x << sh)); // bits 0..(i&31)
}

// The same for 2 <= n < 2^32, in 32-bit arithmetic.
PC_HD uint32_t pc_pi_lookup32(const uint2 *tab, uint32_t n)
{
    const uint32_t i = (n - 1) >> 1;
    const uint2 e = tab[i >> 5];
    return 1u + e.y + (uint32_t)__builtin_popcount(e.x << (31u - (i & 31)));
}

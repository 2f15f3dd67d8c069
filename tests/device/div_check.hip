// Device check of the quotient helpers the kernels use (pc_device.h), run on
// the GPU itself: the fp64 reciprocal with Newton steps (pc_rcp_f64), the
// varying-divisor quotients pc_quot32, pc_quot31, pc_quot31r (stored
// reciprocal) and pc_quot_in, the fp64 division quotient pc_div_small_q, the
// reciprocal division pc_div, and the helpers of x above 2^64: pc_div_wide32
// and pc_div_u128_32 (long division of a 128-bit dividend), pc_div_wide,
// pc_div_small_qd and pc_quot_in64 (a 128-bit dividend given as its low word
// and its value in fp64) and pc_isqrt_wide.  Every result q
// is checked exactly, without any division: either n is built as q d + r
// with r < d, or q d <= n < (q + 1) d is tested in 128-bit arithmetic.
// Inputs: pairs drawn from a counter-based generator (splitmix64 of the pair
// index and a seed), shaped to cover each helper's whole domain (divisors of
// every bit length, quotients up to the helper's bound, remainders 0 and
// d - 1), plus edge pairs.
//
// Built as a shared library by the package build; the test calls
// pc_div_check() through ctypes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pc_device.h"

namespace {

__device__ __forceinline__ uint64_t splitmix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ bool exact(uint64_t n, uint64_t d, uint64_t q)
{
    const pc_u128 lo = (pc_u128)q * d, hi = lo + d;
    return lo <= n && (pc_u128)n < hi;
}

// fails[k]: failures of helper k; first[k]: the first failing pair index
__global__ void k_div_check(uint64_t n_pairs, uint64_t seed, unsigned long long *fails,
                            unsigned long long *first)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pairs; i += stride) {
        const uint64_t r0 = splitmix(seed ^ (i * 4 + 0)), r1 = splitmix(seed ^ (i * 4 + 1));
        const uint64_t r2 = splitmix(seed ^ (i * 4 + 2)), r3 = splitmix(seed ^ (i * 4 + 3));
        // a 32-bit divisor of random bit length (>= 1)
        uint32_t d = (uint32_t)(r0 >> (32 + (r1 & 31)));
        if (d == 0)
            d = 1;
        const uint32_t rm = (r1 >> 8) & 3; // remainder: 0, d - 1 or random
        auto rem = [&](uint64_t r) -> uint64_t {
            return rm == 0 ? 0 : rm == 1 ? d - 1 : (uint64_t)(uint32_t)r % d;
        };
        // quotients below 2^bits with q d + (d - 1) < 2^64: at most 63 - bitlen(d) bits
        const uint32_t lb = 32u - (uint32_t)__builtin_clz(d);
        auto qcap = [&](uint32_t bits) -> uint64_t {
            const uint32_t k = bits < 63u - lb ? bits : 63u - lb;
            return (1ull << k) - 1;
        };
        // pc_quot32: any n < 2^64 whose quotient is below 2^32 - 1
        {
            const uint64_t q = (r2 >> (32 + ((r1 >> 16) & 31))) % 0xFFFFFFFEull; // < 2^32 - 2
            const uint64_t n = q * d + rem(r3);
            const uint32_t got = pc_quot32(n, (double)n, d);
            if (!exact(n, d, got)) {
                atomicAdd(&fails[0], 1ull);
                atomicMin(&first[0], (unsigned long long)i);
            }
        }
        // pc_quot_in: quotient < 2^47 against a window [base, base + span)
        {
            const uint64_t q = (r2 >> (17 + ((r1 >> 24) & 31))) & qcap(47);
            const uint64_t n = q * d + rem(r3); // floor(n / d) = q
            const uint32_t span = 1u + (uint32_t)(r3 >> 35);            // <= 2^29
            const int64_t shift = (int64_t)((r0 >> 3) & 7) - 3;          // window near q
            int64_t b = (q > (uint64_t)span ? (int64_t)(q - span / 2) : 0) + shift;
            const uint64_t base = b < 0 ? 0 : (uint64_t)b;
            uint32_t off = 0xFFFFFFFFu;
            const bool in = pc_quot_in(n, (double)n, d, base, span, &off);
            const bool want_in = q >= base && q < base + span;
            if (in != want_in || (in && base + off != q)) {
                atomicAdd(&fails[1], 1ull);
                atomicMin(&first[1], (unsigned long long)i);
            }
        }
        // pc_div_small_q: quotient < 2^50
        {
            const uint64_t q = (r2 >> (14 + ((r1 >> 40) & 31))) & qcap(50);
            const uint64_t n = q * d + rem(r3);
            if (!exact(n, d, pc_div_small_q(n, d))) {
                atomicAdd(&fails[2], 1ull);
                atomicMin(&first[2], (unsigned long long)i);
            }
        }
        // pc_div: any n, any 64-bit divisor of random bit length, by its reciprocal
        {
            uint64_t D = r3 >> ((r1 >> 48) & 63);
            if (D == 0)
                D = 1;
            const uint64_t n = r2;
            if (!exact(n, D, pc_div(n, D, pc_recip(D)))) {
                atomicAdd(&fails[3], 1ull);
                atomicMin(&first[3], (unsigned long long)i);
            }
        }
        // pc_rcp_f64: relative error below 2^-49 for every 32-bit divisor
        {
            const double r = pc_rcp_f64(d);
            const double e = __builtin_fabs(__builtin_fma(r, (double)d, -1.0));
            if (!(e < 0x1p-49)) {
                atomicAdd(&fails[4], 1ull);
                atomicMin(&first[4], (unsigned long long)i);
            }
        }
        // pc_quot31r / pc_quot31: divisors below 2^31, quotients below 2^32 - 1
        {
            const uint32_t d31 = d >> 1 ? d >> 1 : 1u;
            const uint64_t q = (r2 >> (32 + ((r1 >> 16) & 31))) % 0xFFFFFFFEull;
            const uint64_t rr = rm == 0 ? 0 : rm == 1 ? d31 - 1 : (uint64_t)(uint32_t)r3 % d31;
            const uint64_t n = q * d31 + rr;
            if (!exact(n, d31, pc_quot31r(n, (double)n, d31, 1.0 / (double)d31))) {
                atomicAdd(&fails[5], 1ull);
                atomicMin(&first[5], (unsigned long long)i);
            }
            if (!exact(n, d31, pc_quot31(n, (double)n, d31))) {
                atomicAdd(&fails[6], 1ull);
                atomicMin(&first[6], (unsigned long long)i);
            }
        }
        // pc_div_wide32: x = hi 2^64 + lo with hi < d
        {
            const uint64_t hi = r2 % d, lo = r3;
            uint32_t rem = 0xFFFFFFFFu;
            const uint64_t q = pc_div_wide32(hi, lo, d, &rem);
            const pc_u128 x = ((pc_u128)hi << 64) | lo;
            if (rem >= d || (pc_u128)q * d + rem != x) {
                atomicAdd(&fails[7], 1ull);
                atomicMin(&first[7], (unsigned long long)i);
            }
        }
        // pc_div_wide: quotient below 2^64, divisor below 2^46, x up to 2^110
        // given as its low word and its fp64 value
        {
            uint64_t D = r0 >> (18 + ((r1 >> 32) & 63) % 46);
            if (D == 0)
                D = 1;
            const uint64_t q = r2 >> ((r1 >> 56) & 63);
            const uint64_t rr = rm == 0 ? 0 : rm == 1 ? D - 1 : r3 % D;
            const pc_u128 x = (pc_u128)q * D + rr;
            if (pc_div_wide((uint64_t)x, (double)x, D) != q) {
                atomicAdd(&fails[8], 1ull);
                atomicMin(&first[8], (unsigned long long)i);
            }
        }
        // pc_quot_in64: divisors in [2^32, 2^40), quotient < 2^47, x beyond 2^64
        {
            const uint64_t D = (1ull << 32) | (r0 >> (24 + (r1 & 7)));
            const uint64_t q = (r2 >> (17 + ((r1 >> 24) & 31))) & ((1ull << 47) - 1);
            const uint64_t rr = rm == 0 ? 0 : rm == 1 ? D - 1 : r3 % D;
            const pc_u128 x = (pc_u128)q * D + rr;
            const uint32_t span = 1u + (uint32_t)(r3 >> 35);
            const int64_t shift = (int64_t)((r0 >> 3) & 7) - 3;
            int64_t b = (q > (uint64_t)span ? (int64_t)(q - span / 2) : 0) + shift;
            const uint64_t base = b < 0 ? 0 : (uint64_t)b;
            uint32_t off = 0xFFFFFFFFu;
            const bool in = pc_quot_in64((uint64_t)x, (double)x, D, base, span, &off);
            const bool want_in = q >= base && q < base + span;
            if (in != want_in || (in && base + off != q)) {
                atomicAdd(&fails[9], 1ull);
                atomicMin(&first[9], (unsigned long long)i);
            }
        }
        // pc_div_u128_32: any x below 2^128
        {
            const uint64_t hi = r2 >> ((r1 >> 8) & 63), lo = r3;
            uint64_t qh = 0;
            uint32_t rem = 0xFFFFFFFFu;
            const uint64_t ql = pc_div_u128_32(hi, lo, d, &qh, &rem);
            const pc_u128 x = ((pc_u128)hi << 64) | lo, q = ((pc_u128)qh << 64) | ql;
            if (rem >= d || q * d + rem != x) {
                atomicAdd(&fails[10], 1ull);
                atomicMin(&first[10], (unsigned long long)i);
            }
        }
        // pc_div_small_qd: quotient below 2^50, x up to 2^82 as its low word and fp64 value
        {
            const uint64_t q = (r2 >> (14 + ((r1 >> 40) & 31))) & ((1ull << 50) - 1);
            const pc_u128 x = (pc_u128)q * d + rem(r3);
            if (pc_div_small_qd((uint64_t)x, (double)x, d) != q) {
                atomicAdd(&fails[11], 1ull);
                atomicMin(&first[11], (unsigned long long)i);
            }
        }
        // pc_isqrt_wide: below 2^80 (X_b <= 2^72 in the leaf set-up)
        {
            const uint64_t hi = r2 >> (48 + ((r1 >> 16) & 15)), lo = r3;
            const pc_u128 n = ((pc_u128)hi << 64) | lo;
            const pc_u128 r = pc_isqrt_wide(hi, lo);
            if (!(r * r <= n && (r + 1) * (r + 1) > n)) {
                atomicAdd(&fails[12], 1ull);
                atomicMin(&first[12], (unsigned long long)i);
            }
        }
    }
}

// Edge pairs: divisors 1, 2, 3, 2^31 - 1, 2^32 - 1 and quotients at the ends
// of each helper's domain.
__global__ void k_div_edges(unsigned long long *fails)
{
    const uint32_t ds[] = {1u, 2u, 3u, 5u, 30029u, 65536u, 2147483647u, 2147483648u,
                           4294967291u, 4294967295u};
    const uint32_t d = ds[threadIdx.x % 10];
    const uint64_t qs32[] = {0, 1, 2, 0xFFFFFFFCull, 0xFFFFFFFDull};
    const uint64_t rs[2] = {0, (uint64_t)d - 1};
    for (uint64_t q : qs32)
        for (uint64_t r : rs) {
            const uint64_t n = q * d + r;
            if (!exact(n, d, pc_quot32(n, (double)n, d)))
                atomicAdd(&fails[0], 1ull);
        }
    const uint64_t qs50[] = {0, 1, (1ull << 47) - 1, (1ull << 50) - 1};
    for (uint64_t q : qs50)
        for (uint64_t r : rs) {
            if ((((pc_u128)q * d + r) >> 64) != 0)
                continue; // beyond 2^64
            const uint64_t n = q * d + r;
            if (!exact(n, d, pc_div_small_q(n, d)))
                atomicAdd(&fails[2], 1ull);
            if (q < (1ull << 47)) {
                uint32_t off = 0;
                if (!pc_quot_in(n, (double)n, d, q, 1, &off) || off != 0)
                    atomicAdd(&fails[1], 1ull);
                if (q + 1 < (1ull << 47) && pc_quot_in(n, (double)n, d, q + 1, 5, &off))
                    atomicAdd(&fails[1], 1ull);
            }
        }
    const uint64_t ns[] = {0, 1, ~0ull, ~0ull - 1, 1ull << 63, (1ull << 63) - 1,
                           11529215046068469760ull, 1000000000000000000ull};
    for (uint64_t n : ns) {
        const uint64_t D = (uint64_t)d * (threadIdx.x / 10 + 1);
        if (!exact(n, D, pc_div(n, D, pc_recip(D))))
            atomicAdd(&fails[3], 1ull);
    }
}

} // namespace

// Runs n_pairs random pairs (seeded) and the edge pairs on the current device;
// fails_out[0..12] = failures of pc_quot32, pc_quot_in, pc_div_small_q, pc_div,
// pc_rcp_f64, pc_quot31r, pc_quot31, pc_div_wide32, pc_div_wide,
// pc_quot_in64, pc_div_u128_32, pc_div_small_qd, pc_isqrt_wide; first_out the
// first failing pair index of each (or ~0).
// Returns 0, or the HIP error code.
extern "C" int pc_div_check(uint64_t n_pairs, uint64_t seed, uint64_t *fails_out,
                            uint64_t *first_out)
{
    constexpr int NH = 13;
    unsigned long long *d = nullptr;
    hipError_t e = hipMalloc(&d, 2 * NH * sizeof(unsigned long long));
    if (e != hipSuccess)
        return (int)e;
    unsigned long long init[2 * NH];
    for (int k = 0; k < NH; k++) {
        init[k] = 0;
        init[NH + k] = ~0ull;
    }
    e = hipMemcpy(d, init, sizeof init, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        k_div_check<<<4096, 256>>>(n_pairs, seed, d, d + NH);
        k_div_edges<<<1, 640>>>(d);
        e = hipDeviceSynchronize();
    }
    if (e == hipSuccess)
        e = hipMemcpy(init, d, sizeof init, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess)
        return (int)e;
    for (int k = 0; k < NH; k++) {
        fails_out[k] = init[k];
        first_out[k] = init[NH + k];
    }
    return 0;
}

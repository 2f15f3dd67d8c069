// Device comparison of two ways to read pi(u) for u <= Y, the lookups of the
// easy leaves:
//  * the bitmap the library uses: one 8-byte entry per 64 integers {bits of
//    its 32 odd integers, odd primes below the entry}; pi(u) is one read and
//    a masked popcount;
//  * the sampled table of the paper's Section 2.1: pi(j L) for every multiple
//    of L = floor(log2 Y) (4 bytes per L integers) beside the table of
//    primes; pi(u) starts from pi(L floor(u / L)) and steps through
//    p_{k+1}, p_{k+2}, ... while they are <= u (about L / ln u steps).
// Both kernels read the same query array and write pi(u) per query; the test
// compares the outputs with each other and with a host count.
//
// Built as a shared library by the package build; the test calls
// pc_pi_table_bench() through ctypes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pc_device.h"

namespace {

__global__ void k_bitmap(const uint2 *tab, const uint32_t *u, uint64_t n, uint32_t *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = pc_pi_lookup32(tab, u[i]);
}

// q = floor(v / L) as the high word of v * m, m = ceil(2^32 / L): exact for
// v < 2^32 / (L - 1), far above every u here
__global__ void k_sampled(const uint32_t *samp, uint32_t m, const uint32_t *primes,
                          const uint32_t *u, uint64_t n, uint32_t *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t v = u[i];
        uint32_t k = samp[__umulhi(v, m)];
        while (primes[k + 1] <= v)
            k++;
        out[i] = k;
    }
}

template <typename F> float timed(F &&launch, uint32_t reps)
{
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    launch(); // warm
    (void)hipEventRecord(a, 0);
    for (uint32_t r = 0; r < reps; r++)
        launch();
    (void)hipEventRecord(b, 0);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / (float)reps;
}

} // namespace

// tab: n_tab bitmap entries; samp: n_samp values pi(j L), m = ceil(2^32 / L);
// primes: n_primes values, 1-based (primes[1] = 2), ending with a prime
// above every query; u: n_u queries, 2 <= u.  Writes pi per query of each
// method and the mean kernel time over reps launches.  Returns 0 or the HIP
// error code.
extern "C" int pc_pi_table_bench(const uint2 *tab, uint64_t n_tab, const uint32_t *samp,
                                 uint64_t n_samp, uint32_t m, const uint32_t *primes,
                                 uint64_t n_primes, const uint32_t *u, uint64_t n_u,
                                 uint32_t reps, uint32_t *out_tab, uint32_t *out_samp,
                                 float *ms_tab, float *ms_samp)
{
    void *d_tab = nullptr, *d_samp = nullptr, *d_primes = nullptr, *d_u = nullptr;
    void *d_o1 = nullptr, *d_o2 = nullptr;
    hipError_t e = hipSuccess;
    auto put = [&](void **d, const void *h, size_t bytes) {
        if (e == hipSuccess)
            e = hipMalloc(d, bytes);
        if (e == hipSuccess)
            e = hipMemcpy(*d, h, bytes, hipMemcpyHostToDevice);
    };
    put(&d_tab, tab, n_tab * 8);
    put(&d_samp, samp, n_samp * 4);
    put(&d_primes, primes, n_primes * 4);
    put(&d_u, u, n_u * 4);
    if (e == hipSuccess)
        e = hipMalloc(&d_o1, n_u * 4);
    if (e == hipSuccess)
        e = hipMalloc(&d_o2, n_u * 4);
    if (e == hipSuccess) {
        const uint32_t grid = 4096, block = 256;
        *ms_tab = timed(
            [&] {
                k_bitmap<<<grid, block>>>((const uint2 *)d_tab, (const uint32_t *)d_u, n_u,
                                          (uint32_t *)d_o1);
            },
            reps);
        *ms_samp = timed(
            [&] {
                k_sampled<<<grid, block>>>((const uint32_t *)d_samp, m, (const uint32_t *)d_primes,
                                           (const uint32_t *)d_u, n_u, (uint32_t *)d_o2);
            },
            reps);
        e = hipDeviceSynchronize();
    }
    if (e == hipSuccess)
        e = hipMemcpy(out_tab, d_o1, n_u * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(out_samp, d_o2, n_u * 4, hipMemcpyDeviceToHost);
    for (void *p : {d_tab, d_samp, d_primes, d_u, d_o1, d_o2})
        if (p)
            (void)hipFree(p);
    return (int)e;
}

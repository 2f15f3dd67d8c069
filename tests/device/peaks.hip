// Micro-benchmarks of this GPU's peaks for the sieve's rooflines:
//  * LDS atomic AND with return, the sieve's crossing, on a workgroup's
//    bitmap of 2^13 words padded by one word per 16 (the sieve's layout),
//    in three address patterns: consecutive words (each lane its own bank),
//    the crossing pattern (lane l at bit f + l p of an odd stride p, so words
//    p / 32 apart, p and f changing every step), and pseudo-random words;
//  * 64-bit multiply-high, the core of the reciprocal divisions, as four
//    independent chains per thread;
//  * a device-to-device copy (HBM), counting bytes read plus written.
// Every kernel's result is written out so that no work is dropped.  Built as
// a shared library by the package build; the test calls pc_peaks() through
// ctypes.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint32_t PK_T = 512;          // threads per workgroup, as the sieve's
constexpr uint32_t PK_NW = 1u << 13;    // bitmap words
constexpr uint32_t PK_NWP = PK_NW + PK_NW / 16;

__global__ __launch_bounds__(PK_T) void k_lds(uint32_t iters, uint32_t mode, uint32_t *out)
{
    __shared__ uint32_t bm[PK_NWP];
    for (uint32_t w = threadIdx.x; w < PK_NWP; w += PK_T)
        bm[w] = ~0u;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t h = (blockIdx.x * PK_T + threadIdx.x) * 2654435761u + 1u; // per-lane state
    uint32_t acc = 0;
    for (uint32_t i = 0; i < iters; i++) {
        uint32_t word;
        if (mode == 0) {
            word = ((i * 64u + wv * 1024u) + lane) & (PK_NW - 1);
        } else if (mode == 1) {
            const uint32_t p = 17u + 2u * ((i * 7u + wv * 13u) & 1023u); // odd, 17 .. 2063
            const uint32_t f = (i * 131u + wv * 4099u) & 8191u;
            word = ((f + lane * p) >> 5) & (PK_NW - 1);
        } else {
            h ^= h << 13;
            h ^= h >> 17;
            h ^= h << 5;
            word = h & (PK_NW - 1);
        }
        const uint32_t sh = (i + lane) & 31u;
        const uint32_t old = __hip_atomic_fetch_and(&bm[word + (word >> 4)], ~(1u << sh),
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        acc += (old >> sh) & 1u;
    }
    out[blockIdx.x * PK_T + threadIdx.x] = acc;
}

__global__ __launch_bounds__(PK_T) void k_mulhi(uint32_t iters, uint64_t *out)
{
    const uint64_t g = blockIdx.x * PK_T + threadIdx.x;
    uint64_t x0 = g * 0x9E3779B97F4A7C15ull + 1, x1 = x0 ^ 0xD1B54A32D192ED03ull;
    uint64_t x2 = x0 + 0xABCDEF12345ull, x3 = x1 * 3u + 7u;
    const uint64_t c0 = 0xF1357AEA2E62A9C5ull, c1 = 0xC6A4A7935BD1E995ull;
    const uint64_t c2 = 0x9FB21C651E98DF25ull, c3 = 0xE7037ED1A0B428DBull;
    for (uint32_t i = 0; i < iters; i++) {
        x0 = __umul64hi(x0, c0) + i;
        x1 = __umul64hi(x1, c1) + i;
        x2 = __umul64hi(x2, c2) + i;
        x3 = __umul64hi(x3, c3) + i;
    }
    out[g] = x0 ^ x1 ^ x2 ^ x3;
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

// Measured peaks: lds[3] atomic ANDs with return per second (consecutive,
// crossing pattern, random words), mulhi 64-bit multiply-highs per second,
// copy_bps bytes read plus written per second by a device-to-device copy of
// copy_bytes.  blocks: workgroups of each kernel (a few per CU).  Returns 0 or
// the HIP error code.
extern "C" int pc_peaks(uint32_t blocks, uint32_t iters, uint64_t copy_bytes, double *lds,
                        double *mulhi, double *copy_bps)
{
    void *d_out = nullptr, *d_a = nullptr, *d_b = nullptr;
    hipError_t e = hipMalloc(&d_out, (size_t)blocks * PK_T * 8);
    if (e == hipSuccess)
        e = hipMalloc(&d_a, copy_bytes);
    if (e == hipSuccess)
        e = hipMalloc(&d_b, copy_bytes);
    if (e == hipSuccess)
        e = hipMemset(d_a, 1, copy_bytes);
    if (e == hipSuccess) {
        const double lanes = (double)blocks * PK_T;
        for (uint32_t mode = 0; mode < 3; mode++) {
            const float ms = timed(
                [&] { k_lds<<<blocks, PK_T>>>(iters, mode, (uint32_t *)d_out); }, 5);
            lds[mode] = lanes * iters / (ms * 1e-3);
        }
        const float ms = timed([&] { k_mulhi<<<blocks, PK_T>>>(iters, (uint64_t *)d_out); }, 5);
        *mulhi = 4.0 * lanes * iters / (ms * 1e-3);
        const float mc = timed(
            [&] { (void)hipMemcpyAsync(d_b, d_a, copy_bytes, hipMemcpyDeviceToDevice, 0); }, 5);
        *copy_bps = 2.0 * (double)copy_bytes / (mc * 1e-3);
        e = hipDeviceSynchronize();
    }
    for (void *p : {d_out, d_a, d_b})
        if (p)
            (void)hipFree(p);
    return (int)e;
}

// Host-side check of the integer helpers in pc_device.h: exact division by a
// precomputed reciprocal, the fp64-estimate divisions, integer roots and the
// pi-table lookup, against plain 128-bit arithmetic and a trial-division sieve.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "pc_device.h"

static int fails = 0;
#define CHECK(cond, ...)                                                                     \
    do {                                                                                     \
        if (!(cond)) {                                                                       \
            if (fails++ < 20) {                                                              \
                std::printf("FAIL %s:%d ", __FILE__, __LINE__);                              \
                std::printf(__VA_ARGS__);                                                    \
                std::printf("\n");                                                           \
            }                                                                                \
        }                                                                                    \
    } while (0)

int main()
{
    std::mt19937_64 rng(1503);
    const uint64_t edges[] = {0, 1, 2, 3, (1ull << 32) - 1, 1ull << 32, (1ull << 63) - 1,
                              1ull << 63, (1ull << 63) + 1, ~0ull - 1, ~0ull,
                              1000000000000000000ull, 11529215046068469760ull};
    // exhaustive small divisors, edge dividends
    for (uint64_t d = 1; d <= 70000; d++) {
        uint64_t r = pc_recip(d);
        for (uint64_t n : edges)
            CHECK(pc_div(n, d, r) == n / d, "pc_div(%llu, %llu)", (unsigned long long)n,
                  (unsigned long long)d);
        for (int k = 0; k < 8; k++) {
            uint64_t n = rng();
            CHECK(pc_div(n, d, r) == n / d, "pc_div rnd");
            CHECK(pc_div_any(n, (uint32_t)d) == n / d, "pc_div_any(%llu, %llu)",
                  (unsigned long long)n, (unsigned long long)d);
        }
    }
    // random 64-bit divisors (segment bounds) and 32-bit divisors
    for (int i = 0; i < 2000000; i++) {
        uint64_t n = rng(), d = rng() >> (rng() % 64);
        if (d == 0)
            d = 1;
        CHECK(pc_div(n, d, pc_recip(d)) == n / d, "pc_div64");
        uint32_t d32 = (uint32_t)(rng() >> (32 + rng() % 32));
        if (d32 == 0)
            d32 = 1;
        CHECK(pc_div_any(n, d32) == n / d32, "pc_div_any");
        // quotient < 2^50 regime of pc_div_small_q
        uint64_t m = n >> (rng() % 40);
        if (m / d32 < (1ull << 50))
            CHECK(pc_div_small_q(m, d32) == m / d32, "pc_div_small_q(%llu,%u)",
                  (unsigned long long)m, d32);
    }
    for (uint64_t n : edges)
        for (uint32_t d : {1u, 2u, 3u, 17u, 4294967295u, 2147483647u})
            CHECK(pc_div_any(n, d) == n / d, "pc_div_any edge");
    // roots
    for (uint64_t n : edges) {
        uint64_t r = pc_isqrt(n), c = pc_icbrt(n);
        CHECK((pc_u128)r * r <= n && (pc_u128)(r + 1) * (r + 1) > n, "isqrt");
        CHECK((pc_u128)c * c * c <= n && (pc_u128)(c + 1) * (c + 1) * (c + 1) > n, "icbrt");
    }
    for (int i = 0; i < 1000000; i++) {
        uint64_t n = rng() >> (rng() % 64);
        uint64_t r = pc_isqrt(n), c = pc_icbrt(n);
        CHECK((pc_u128)r * r <= n && (pc_u128)(r + 1) * (r + 1) > n, "isqrt rnd");
        CHECK((pc_u128)c * c * c <= n && (pc_u128)(c + 1) * (c + 1) * (c + 1) > n, "icbrt rnd");
    }
    // pi lookup on a table built here by trial division
    const uint64_t N = 1 << 16;
    std::vector<uint2> tab(N / 64 + 1);
    std::vector<int> isp(N + 64, 1);
    isp[0] = isp[1] = 0;
    for (uint64_t i = 2; i < isp.size(); i++)
        for (uint64_t d = 2; d * d <= i; d++)
            if (i % d == 0) {
                isp[i] = 0;
                break;
            }
    uint32_t run = 0;
    for (uint64_t e = 0; e < tab.size(); e++) {
        uint32_t bits = 0;
        for (int j = 0; j < 32; j++)
            if (isp[64 * e + 2 * j + 1])
                bits |= 1u << j;
        tab[e].x = bits;
        tab[e].y = run;
        run += __builtin_popcount(bits);
    }
    uint32_t pi = 0;
    for (uint64_t n = 0; n < N; n++) {
        pi += isp[n];
        CHECK(pc_pi_lookup(tab.data(), n) == pi, "pi(%llu)", (unsigned long long)n);
    }
    std::printf(fails ? "FAILED %d\n" : "OK\n", fails);
    return fails ? 1 : 0;
}

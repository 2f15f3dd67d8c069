// pc_tables.hip -- device tables of the prime-counting library, all built on
// the GPU:
//   * primes p_k (1-based) and an odd-only pi table up to a limit P < 2^32
//     (Section 2.1 of the paper keeps pi(y) and the primes p_b; here pi is a
//     bitmap with a running count per 32 odd numbers, 8 bytes per 64 integers);
//   * 64-bit reciprocals of the primes, for exact division by invariant
//     divisors;
//   * mu(n)*lpf(n) for n <= y (Section 2.2: "p_min(y) mu(y)");
//   * the wheel of size c (Section 4): the odd-only pre-sieve pattern of
//     p_2..p_c and phi(r, c) for r below the primorial Q_c.
#include "pc_block.h"
#include "pc_internal.h"

// ---------------------------------------------------------------------------
// Odd primes below 2^16, by one workgroup (enough to sieve up to 2^32).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_base_primes(uint32_t *base, uint32_t *nbase)
{
    constexpr uint32_t W = 4096, N = 64 * W; // the odd numbers below 2^18
    __shared__ uint32_t bits[W]; // bit j of word w <-> 64w + 2j + 1
    __shared__ uint32_t scr[16];
    const uint32_t t = threadIdx.x;
    for (uint32_t w = t; w < W; w += 1024)
        bits[w] = w == 0 ? 0xFFFFFFFEu : 0xFFFFFFFFu; // 1 is not prime
    __syncthreads();
    // odd q in [3, 511], the odd multiples from q^2 shared by all threads;
    // composite q only repeats its factors' work
    for (uint32_t q = 3; q < 512; q += 2)
        for (uint32_t n = q * q + 2 * q * t; n < N; n += 2 * q * 1024) {
            const uint32_t i = n >> 1;
            atomicAnd(&bits[i >> 5], ~(1u << (i & 31)));
        }
    __syncthreads();
    // thread t owns words 4t .. 4t + 3
    uint32_t w4[4], c = 0;
    for (uint32_t k = 0; k < 4; k++) {
        w4[k] = bits[4 * t + k];
        c += (uint32_t)__builtin_popcount(w4[k]);
    }
    uint32_t total;
    uint32_t off = pc_block_excl_scan<1024>(c, scr, &total);
    for (uint32_t k = 0; k < 4; k++) {
        uint32_t w = w4[k];
        while (w) {
            uint32_t j = __builtin_ctz(w);
            w &= w - 1;
            base[off++] = 64 * (4 * t + k) + 2 * j + 1;
        }
    }
    if (t == 0)
        *nbase = total;
}

// ---------------------------------------------------------------------------
// Segmented odd-only sieve of Eratosthenes over entries [0, nent): entry e
// covers the odd numbers 64e+1 .. 64e+63.  Writes the prime bits into
// tab[e].x and their popcount into cnt[e].  The odd primes 3 .. 31 (the first
// PT_NPRE base primes, over half of all the crossings) are not crossed one
// multiple at a time: each word starts as the AND of their periodic masks,
// chosen by the residue of the word's first odd number modulo each prime.
// ---------------------------------------------------------------------------
#define PT_WORDS 4096 // entries per workgroup: 131072 odd numbers
#define PT_T 1024
#define PT_NPRE 10
namespace {
constexpr uint32_t kPreQ[PT_NPRE] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31};
constexpr uint32_t kPreOff[PT_NPRE + 1] = {0, 3, 8, 15, 26, 39, 56, 75, 98, 127, 158};
// bits of 3 .. 31 in the first word (bit j <-> 2j + 1)
constexpr uint32_t kPrePrimes = (1u << 1) | (1u << 2) | (1u << 3) | (1u << 5) | (1u << 6) |
                                (1u << 8) | (1u << 9) | (1u << 11) | (1u << 14) | (1u << 15);
} // namespace

__global__ __launch_bounds__(PT_T) void k_sieve_pitab(uint64_t nent, const uint32_t *base,
                                                    uint32_t nbase, uint2 *tab, uint32_t *cnt)
{
    __shared__ uint32_t bits[PT_WORDS];
    __shared__ uint32_t first[PT_T]; // start index of each small prime, computed once
    __shared__ uint32_t keep[kPreOff[PT_NPRE]]; // per pre-sieved prime q and residue r
    __shared__ uint32_t res0[PT_NPRE];          // the block's first odd number mod q
    const uint32_t t = threadIdx.x;
    const uint64_t e0 = (uint64_t)blockIdx.x * PT_WORDS;
    if (t < kPreOff[PT_NPRE]) {
        // the word whose first odd number is r mod q keeps bit j unless q | r + 2j
        uint32_t i = 0;
        while (t >= kPreOff[i + 1])
            i++;
        const uint32_t q = kPreQ[i], r = t - kPreOff[i];
        uint32_t w = 0xFFFFFFFFu;
        for (uint32_t j = 0; j < 32; j++)
            if ((r + 2 * j) % q == 0)
                w &= ~(1u << j);
        keep[t] = w;
    }
    if (t < PT_NPRE)
        res0[t] = (uint32_t)((64 * e0 + 1) % kPreQ[t]);
    __syncthreads();
    for (uint32_t i = t; i < PT_WORDS; i += PT_T) {
        uint32_t w = 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t k = 0; k < PT_NPRE; k++) {
            const uint32_t q = kPreQ[k];
            w &= keep[kPreOff[k] + (res0[k] + (64 % q) * i) % q];
        }
        if (e0 == 0 && i == 0)
            w = (w | kPrePrimes) & ~1u; // 3 .. 31 are prime, 1 is not
        bits[i] = w;
    }
    const uint64_t nlo = 64 * e0;                   // first integer covered
    const uint64_t nhi = 64 * (e0 + PT_WORDS) - 1;  // last integer covered
    const uint32_t NBIT = PT_WORDS * 32;
    // bit index (from nlo) of the first odd multiple of q that is >= nlo and >= q^2
    auto start = [&](uint32_t q) -> uint32_t {
        const uint32_t r = (uint32_t)(nlo % q);
        uint64_t m = nlo + (r ? q - r : 0);
        if ((m & 1) == 0)
            m += q;
        if (m < (uint64_t)q * q)
            m = (uint64_t)q * q;
        const uint64_t bi = ((m - 1) >> 1) - (nlo >> 1);
        return bi < NBIT ? (uint32_t)bi : NBIT;
    };
    // small primes (q < 4 PT_T, q^2 <= nhi: a prefix of base[], at most PT_T
    // of them): their starts once per workgroup, then all threads share the
    // multiples of one prime at a time
    const bool small = t < nbase && base[t] < 4 * PT_T && (uint64_t)base[t] * base[t] <= nhi;
    if (small)
        first[t] = start(base[t]);
    const uint32_t nsm = (uint32_t)__syncthreads_count(small);
    // (every block ends at or above 64 PT_WORDS - 1 > 31^2: nsm > PT_NPRE)
    for (uint32_t k = PT_NPRE; k < nsm; k++) {
        const uint32_t q = base[k];
        for (uint32_t i = first[k] + t * q; i < NBIT; i += PT_T * q)
            atomicAnd(&bits[i >> 5], ~(1u << (i & 31)));
    }
    // large primes: one lane per prime
    for (uint32_t j = nsm + t; j < nbase; j += PT_T) {
        const uint32_t q = base[j];
        if ((uint64_t)q * q > nhi)
            continue;
        for (uint32_t i = start(q); i < NBIT; i += q)
            atomicAnd(&bits[i >> 5], ~(1u << (i & 31)));
    }
    __syncthreads();
    for (uint32_t i = t; i < PT_WORDS; i += PT_T) {
        uint64_t e = e0 + i;
        if (e < nent) {
            tab[e].x = bits[i];
            cnt[e] = (uint32_t)__builtin_popcount(bits[i]);
        }
    }
}

// ---------------------------------------------------------------------------
// Exclusive scans (reduce, scan of block sums, down-sweep).
// ---------------------------------------------------------------------------
#define SC_T 256
#define SC_ITEMS 16
#define SC_TILE (SC_T * SC_ITEMS)

template <typename T>
__global__ __launch_bounds__(SC_T) void k_scan_reduce(const T *in, uint64_t n, T *bsum)
{
    __shared__ T scr[SC_T / 64];
    uint64_t base = (uint64_t)blockIdx.x * SC_TILE;
    T s = 0;
    for (uint32_t i = 0; i < SC_ITEMS; i++) {
        uint64_t j = base + (uint64_t)i * SC_T + threadIdx.x;
        if (j < n)
            s += in[j];
    }
    s = pc_block_sum<SC_T>(s, scr);
    if (threadIdx.x == 0)
        bsum[blockIdx.x] = s;
}

// one workgroup scans the block sums in place; *total receives the grand total
template <typename T>
__global__ __launch_bounds__(SC_T) void k_scan_top(T *bsum, uint64_t nb, T *total)
{
    __shared__ T scr[SC_T / 64];
    T run = 0;
    for (uint64_t c0 = 0; c0 < nb; c0 += SC_T) {
        uint64_t j = c0 + threadIdx.x;
        T v = j < nb ? bsum[j] : 0, tot;
        T ex = pc_block_excl_scan<SC_T>(v, scr, &tot);
        if (j < nb)
            bsum[j] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0 && total)
        *total = run;
}

template <typename T>
__global__ __launch_bounds__(SC_T) void k_scan_down(T *data, uint64_t n, const T *bsum)
{
    __shared__ T scr[SC_T / 64];
    uint64_t base = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_ITEMS;
    T v[SC_ITEMS];
    T s = 0;
    for (uint32_t i = 0; i < SC_ITEMS; i++) {
        uint64_t j = base + i;
        v[i] = j < n ? data[j] : 0;
        s += v[i];
    }
    T tot;
    T ex = pc_block_excl_scan<SC_T>(s, scr, &tot) + bsum[blockIdx.x];
    for (uint32_t i = 0; i < SC_ITEMS; i++) {
        uint64_t j = base + i;
        if (j < n)
            data[j] = ex;
        ex += v[i];
    }
}

template <typename T>
static hipError_t scan_excl(T *data, uint64_t n, T *tmp, T *total, hipStream_t s)
{
    uint64_t nb = (n + SC_TILE - 1) / SC_TILE;
    if (nb == 0)
        nb = 1;
    k_scan_reduce<T><<<(uint32_t)nb, SC_T, 0, s>>>(data, n, tmp);
    k_scan_top<T><<<1, SC_T, 0, s>>>(tmp, nb, total);
    k_scan_down<T><<<(uint32_t)nb, SC_T, 0, s>>>(data, n, tmp);
    return hipGetLastError();
}

hipError_t pc_launch_scan_u64(uint64_t *data, uint64_t n, uint64_t *tmp, uint64_t *total,
                              hipStream_t s)
{
    return scan_excl<uint64_t>(data, n, tmp, total, s);
}

// tab[e].y = number of odd primes in entries < e; primes[] filled in order,
// the primes of entries e >= 2^26 (above 2^32) into primes_hi[k - k32], k32
// the index of the first of them.
__global__ void k_pitab_pack(uint64_t nent, uint2 *tab, const uint32_t *pre, uint32_t *primes,
                             uint64_t *primes_hi)
{
    constexpr uint64_t E32 = 1ull << 26;
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) {
        primes[0] = 0;
        primes[1] = 2;
    }
    if (e >= nent)
        return;
    uint32_t off = pre[e];
    uint32_t w = tab[e].x;
    tab[e].y = off;
    uint32_t k = off + 2; // odd prime of rank off is p_{off+2}
    if (e < E32) {
        while (w) {
            uint32_t j = __builtin_ctz(w);
            w &= w - 1;
            primes[k++] = (uint32_t)(64 * e + 2 * j + 1);
        }
    } else {
        const uint32_t k32 = pre[E32] + 2;
        while (w) {
            uint32_t j = __builtin_ctz(w);
            w &= w - 1;
            primes_hi[k++ - k32] = 64 * e + 2 * j + 1;
        }
    }
}

hipError_t pc_launch_pitab(uint64_t nent, const uint32_t *base, uint32_t nbase, uint32_t *bits,
                           uint32_t *cnts, uint2 *pitab, uint32_t *primes, uint64_t *primes_hi,
                           uint32_t *scan_tmp, hipStream_t s)
{
    (void)bits;
    // base primes reach 2^18 (every n < 262147^2 sieved), so the table reaches
    // 2^36 + 2^20; prefix counts are 32-bit (pi(2^37) < 2^32)
    if (nent > (1ull << 30) + (1ull << 14) || (nent > (1ull << 26) && !primes_hi))
        return hipErrorInvalidValue;
    uint32_t nblk = (uint32_t)((nent + PT_WORDS - 1) / PT_WORDS);
    k_sieve_pitab<<<nblk, PT_T, 0, s>>>(nent, base, nbase, pitab, cnts);
    hipError_t e = scan_excl<uint32_t>(cnts, nent, scan_tmp, (uint32_t *)nullptr, s);
    if (e != hipSuccess)
        return e;
    k_pitab_pack<<<(uint32_t)((nent + 255) / 256), 256, 0, s>>>(nent, pitab, cnts, primes,
                                                                 primes_hi);
    return hipGetLastError();
}

hipError_t pc_launch_base_primes(uint32_t *base, uint32_t *nbase, hipStream_t s)
{
    k_base_primes<<<1, 1024, 0, s>>>(base, nbase);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reciprocals recip[k] = floor((2^64-1) / p_k) and rcpd[k] = 1/p_k (IEEE
// double, correctly rounded), k in [1, n].
// ---------------------------------------------------------------------------
__global__ void k_recip(const uint32_t *primes, uint64_t *recip, double *rcpd, uint32_t n)
{
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) {
        recip[0] = 0;
        rcpd[0] = 0.0;
    }
    if (k >= 1 && k <= n) {
        recip[k] = pc_recip(primes[k]);
        rcpd[k] = 1.0 / (double)primes[k];
    }
}

hipError_t pc_launch_recip(const uint32_t *primes, uint64_t *recip, double *rcpd, uint32_t n,
                           hipStream_t s)
{
    k_recip<<<(n + 256) / 256, 256, 0, s>>>(primes, recip, rcpd, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// mu(n)*lpf(n) for n <= ymax by a segmented factor sieve.  Each workgroup owns
// MF_N consecutive n and applies every prime p <= sqrt(ymax) (all below 2^16)
// to them; a cofactor left above 1 is one prime > sqrt(ymax).
//
// Per n three words, each updated only by LDS atomics that commute, so that
// the primes can be applied in any order and by any threads with no barrier
// between them: the least prime factor (atomic min), the parity of the number
// of distinct small prime factors in bit 0 and "some p^2 divides n" in bit 1
// (atomic xor, or), and the product of the distinct small prime factors
// (compare-and-swap multiply; it stays <= n < 2^31).  The first MF_PS primes,
// whose multiples are dense, are shared by all threads of the workgroup; each
// larger prime (at most MF_N / p_(MF_PS+1) < 16 multiples, and at most one
// multiple of p^2) belongs to one thread.
// ---------------------------------------------------------------------------
#define MF_N 4096
#define MF_T 512
#define MF_PS 64

__global__ __launch_bounds__(MF_T) void k_mulpf(const uint32_t *primes, uint32_t nsmall,
                                               uint64_t ymax, int32_t *out)
{
    __shared__ uint32_t lp[MF_N], fl[MF_N], prod[MF_N];
    __shared__ uint32_t f1[MF_PS], f2[MF_PS]; // first multiples of p and p^2 in the block
    const uint32_t t = threadIdx.x;
    const uint32_t n0 = blockIdx.x * MF_N; // ymax < 2^31: every n fits 32 bits
    for (uint32_t i = t; i < MF_N; i += MF_T) {
        lp[i] = 0xFFFFFFFFu;
        fl[i] = 0;
        prod[i] = 1;
    }
    // offsets from n0 of the first multiples of p and of p^2 (0xFFFFFFFF:
    // p^2 has none in the block)
    auto offsets = [&](uint32_t p, uint32_t *o1, uint32_t *o2) {
        const uint32_t r = n0 % p;
        *o1 = r ? p - r : 0;
        *o2 = 0xFFFFFFFFu;
        const uint64_t pp = (uint64_t)p * p;
        if (pp < (uint64_t)n0 + MF_N) { // then pp < 2^32
            const uint32_t r2 = n0 % (uint32_t)pp;
            *o2 = r2 ? (uint32_t)pp - r2 : 0;
        }
    };
    const uint32_t ns = min(nsmall, (uint32_t)MF_PS);
    if (t < ns)
        offsets(primes[1 + t], &f1[t], &f2[t]);
    __syncthreads();
    auto mark = [&](uint32_t i, uint32_t p) {
        atomicMin(&lp[i], p);
        atomicXor(&fl[i], 1u);
        uint32_t old = prod[i];
        for (;;) {
            const uint32_t seen = atomicCAS(&prod[i], old, old * p);
            if (seen == old)
                break;
            old = seen;
        }
    };
    for (uint32_t k = 0; k < ns; k++) {
        const uint32_t p = primes[1 + k];
        for (uint32_t i = f1[k] + t * p; i < MF_N; i += MF_T * p)
            mark(i, p);
        const uint32_t o2 = f2[k];
        if (o2 != 0xFFFFFFFFu) {
            const uint64_t pp = (uint64_t)p * p;
            for (uint64_t i = o2 + (uint64_t)t * pp; i < MF_N; i += MF_T * pp)
                atomicOr(&fl[i], 2u);
        }
    }
    for (uint32_t k = ns + 1 + t; k <= nsmall; k += MF_T) {
        const uint32_t p = primes[k];
        uint32_t o1, o2;
        offsets(p, &o1, &o2);
        for (uint32_t i = o1; i < MF_N; i += p)
            mark(i, p);
        if (o2 < MF_N)
            atomicOr(&fl[o2], 2u);
    }
    __syncthreads();
    for (uint32_t i = t; i < MF_N; i += MF_T) {
        uint64_t n = (uint64_t)n0 + i;
        if (n > ymax)
            continue;
        int32_t v;
        if (n == 0) {
            v = 0;
        } else if (n == 1) {
            v = 0x7FFFFFFF;
        } else if (fl[i] & 2u) {
            v = 0;
        } else {
            int32_t m = (fl[i] & 1u) ? -1 : 1;
            uint32_t l = lp[i];
            if (prod[i] < n) { // one prime factor above sqrt(ymax)
                m = -m;
                if (l == 0xFFFFFFFFu)
                    l = (uint32_t)n / prod[i];
            }
            v = m * (int32_t)l;
        }
        out[n] = v;
    }
}

// *out += the number of nonzero entries of a[1..n] (a consistency check of the
// mu*lpf table: those are the squarefree n <= ymax).
__global__ __launch_bounds__(256) void k_count_nonzero(const int32_t *a, uint64_t n,
                                                      unsigned long long *out)
{
    __shared__ unsigned long long scr[4];
    unsigned long long c = 0;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = 1 + (uint64_t)blockIdx.x * 256 + threadIdx.x; i <= n; i += stride)
        c += a[i] != 0 ? 1u : 0u;
    c = pc_block_sum<256>(c, scr);
    if (threadIdx.x == 0)
        atomicAdd(out, c);
}

hipError_t pc_launch_count_nonzero(const int32_t *a, uint64_t n, unsigned long long *out,
                                   hipStream_t s)
{
    k_count_nonzero<<<1024, 256, 0, s>>>(a, n, out);
    return hipGetLastError();
}

hipError_t pc_launch_mulpf(const uint32_t *primes, uint32_t nsmall, uint64_t ymax, int32_t *mulpf,
                           hipStream_t s)
{
    if (ymax >= (1ull << 31)) // k_mulpf's 32-bit arithmetic
        return hipErrorInvalidValue;
    uint32_t nblk = (uint32_t)(ymax / MF_N + 1);
    k_mulpf<<<nblk, MF_T, 0, s>>>(primes, nsmall, ymax, mulpf);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wheel of size c: pattern bit j <-> 2j+1 coprime to p_2..p_c, j < period+64;
// phitab[r] = phi(r, c) for 0 <= r < Q_c.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_wheel(uint32_t c, const uint32_t *primes,
                                              uint32_t *pattern, uint32_t pattern_words,
                                              uint32_t *phitab, uint32_t *wres)
{
    __shared__ uint32_t scr[16];
    const uint32_t t = threadIdx.x;
    uint32_t P[8];
    uint32_t Q = 1;
    for (uint32_t i = 1; i <= c; i++) {
        P[i - 1] = primes[i];
        Q *= primes[i];
    }
    for (uint32_t w = t; w < pattern_words; w += 1024) {
        uint32_t word = 0;
        for (uint32_t j = 0; j < 32; j++) {
            uint32_t n = 2 * (32 * w + j) + 1;
            bool ok = true;
            for (uint32_t i = 1; i < c; i++)
                ok = ok && (n % P[i] != 0);
            word |= (ok ? 1u : 0u) << j;
        }
        pattern[w] = word;
    }
    // phi(r, c): each thread a contiguous chunk of r
    uint32_t per = (Q + 1023) / 1024;
    uint32_t r0 = t * per, r1 = min(Q, r0 + per);
    uint32_t local = 0;
    for (uint32_t r = max(r0, 1u); r < r1; r++) {
        bool ok = true;
        for (uint32_t i = 0; i < c; i++)
            ok = ok && (r % P[i] != 0);
        local += ok;
    }
    uint32_t total;
    uint32_t run = pc_block_excl_scan<1024>(local, scr, &total);
    for (uint32_t r = r0; r < r1; r++) {
        if (r >= 1) {
            bool ok = true;
            for (uint32_t i = 0; i < c; i++)
                ok = ok && (r % P[i] != 0);
            run += ok;
        }
        phitab[r] = run;
    }
    __syncthreads();
    // the residues prime to p_1..p_c in order: r is number phi(r, c) - 1
    for (uint32_t r = max(r0, 1u); r < r1; r++) {
        bool ok = true;
        for (uint32_t i = 0; i < c; i++)
            ok = ok && (r % P[i] != 0);
        if (ok)
            wres[phitab[r] - 1] = r;
    }
}

hipError_t pc_launch_wheel(uint32_t c, const uint32_t *primes, uint32_t *pattern,
                           uint32_t pattern_words, uint32_t *phitab, uint32_t *wres,
                           hipStream_t s)
{
    k_wheel<<<1, 1024, 0, s>>>(c, primes, pattern, pattern_words, phitab, wres);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small helpers: pi at a few points; X_b = floor(x / p_b).
// ---------------------------------------------------------------------------
__global__ void k_lookup(const uint2 *pitab, const uint64_t *in, uint32_t n, uint64_t *out)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = pc_pi_lookup(pitab, in[i]);
}

hipError_t pc_launch_lookup(const uint2 *pitab, const uint64_t *in, uint32_t n, uint64_t *out,
                            hipStream_t s)
{
    k_lookup<<<(n + 63) / 64, 64, 0, s>>>(pitab, in, n, out);
    return hipGetLastError();
}


// pc_host.hip -- host planner and C ABI of the prime-counting library.
//
// The host validates arguments, picks y, the wheel size c and the segment
// geometry, keeps the shared device tables, cuts the sieve range [1, x/y]
// into windows and tiles, launches the kernels in stream order and reads
// back one small result record.  Every arithmetic step of the method runs
// in the kernels of pc_tables.hip, pc_leaves.hip and pc_sieve.hip.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/picount.h"
#include "pc_internal.h"
#include "pc_alpha_table.h"

namespace {

constexpr int kWheelC = 6;
constexpr uint64_t kSmallX = 1ull << 20; // below this pi(x) is read from the pi table

thread_local std::string t_err;
std::recursive_mutex g_mu;

struct pc_error {
    pc_status st;
    std::string msg;
};

[[noreturn]] void fail(pc_status st, const std::string &msg) { throw pc_error{st, msg}; }

void hipck(hipError_t e, const char *what)
{
    if (e != hipSuccess)
        fail(PC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

std::atomic<size_t> g_dev_bytes{0}, g_dev_peak{0}; // device bytes held, and their peak

hipStream_t g_stream = nullptr;  // the library stream
hipStream_t g_stream2 = nullptr; // easy leaves, concurrent with the sieve (same priority)
hipStream_t g_stream3 = nullptr; // the candidate easy leaves, beside the bands (same priority)

// Completion events of caller-memory batches queued on callers' streams
// (they read the shared tables), and spare events to record the next ones.
std::vector<hipEvent_t> g_async_live, g_async_spare;

void async_wait_all()
{
    for (hipEvent_t e : g_async_live) {
        (void)hipEventSynchronize(e);
        g_async_spare.push_back(e);
    }
    g_async_live.clear();
}

void dfree(DevBuf &b)
{
    if (b.p) {
        async_wait_all(); // kernels queued earlier may still read the buffer
        if (g_stream2)
            (void)hipStreamSynchronize(g_stream2);
        if (g_stream3)
            (void)hipStreamSynchronize(g_stream3);
        if (g_stream)
            (void)hipStreamSynchronize(g_stream);
        (void)hipFree(b.p);
        g_dev_bytes -= b.cap;
    }
    b.p = nullptr;
    b.cap = 0;
}

void ensure(DevBuf &b, size_t bytes, const char *what)
{
    if (bytes == 0)
        bytes = 16;
    if (b.cap >= bytes)
        return;
    dfree(b);
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(PC_ENOMEM, std::string("device allocation of ") + std::to_string(bytes) +
                            " bytes for " + what + " failed");
    }
    b.cap = bytes;
    g_dev_bytes += bytes;
    g_dev_peak = std::max<size_t>(g_dev_peak.load(), g_dev_bytes.load());
}

template <typename T> T *ptr(DevBuf &b) { return static_cast<T *>(b.p); }

// first primes, for the wheel constants only
const uint32_t kFirstPrimes[8] = {0, 2, 3, 5, 7, 11, 13, 17};

struct Tables {
    bool base_ok = false;
    uint32_t nbase = 0;
    DevBuf base, nbase_d;
    DevBuf pitab, primes, primes_hi, cnt_tmp, scan_tmp;
    uint64_t pi_limit = 0; // pi table and primes cover n <= pi_limit
    uint64_t nprimes = 0;
    uint64_t k32 = ~0ull;  // index of the first prime above 2^32 (in primes_hi), if covered
    DevBuf recip, rcpd;
    uint64_t recip_n = 0;
    DevBuf mulpf;
    uint64_t y_limit = 0;
    DevBuf pattern[kWheelC + 1], phitab[kWheelC + 1], wres[kWheelC + 1];
    bool wheel_ok[kWheelC + 1] = {};
    uint32_t pattern_bits[kWheelC + 1] = {}, Qc[kWheelC + 1] = {}, phiQ[kWheelC + 1] = {};
    DevBuf lk_in, lk_out, chk;
    // the first entries of the device pi table, read back for planning the
    // count staircase on the host (pi at isqrt(x / lo): every segment but the
    // first starts at lo >= 2^16, so below 2^24 for x < 2^64 and at most 2^28
    // for x <= 2^72)
    // (pinned host memory, kept across rebuilds: the copy runs at the link's rate)
    uint2 *pi_host = nullptr;
    size_t pi_host_cap = 0;   // entries allocated
    uint64_t pi_host_max = 0; // pi_host answers n <= pi_host_max
};
Tables g_T;

// Pinned host memory for the plan copies of one query (row offsets, scan
// blocks, tile lists, the tile planner's reads): a copy from pageable memory
// goes through the runtime's staging at a few GB/s, one from here at the
// link's rate.  Each copy takes its own stretch, which stays untouched until
// the next query resets the arena after synchronising the library stream, so
// a copy that the stream reaches late still reads what was written for it.
// The chunks are kept from one query to the next, up to 64 MiB (a query near
// 2^72 plans hundreds of MiB of tiles; that memory goes back after it).
struct PinnedArena {
    struct Chunk {
        char *p;
        size_t cap, used;
    };
    std::vector<Chunk> chunks;
    size_t cur = 0;
    void *take(size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        while (cur < chunks.size() && chunks[cur].cap - chunks[cur].used < bytes)
            cur++;
        if (cur == chunks.size()) {
            const size_t cap = std::max<size_t>(bytes, (size_t)8 << 20);
            void *p = nullptr;
            if (hipHostMalloc(&p, cap, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                fail(PC_ENOMEM, "pinned staging memory for the query plan");
            }
            chunks.push_back(Chunk{static_cast<char *>(p), cap, 0});
        }
        Chunk &c = chunks[cur];
        void *r = c.p + c.used;
        c.used += bytes;
        return r;
    }
    void reset()
    {
        size_t total = 0;
        for (Chunk &c : chunks) {
            c.used = 0;
            total += c.cap;
        }
        cur = 0;
        if (total > ((size_t)64 << 20))
            release();
    }
    void release()
    {
        for (Chunk &c : chunks)
            (void)hipHostFree(c.p);
        chunks.clear();
        cur = 0;
    }
};
PinnedArena g_pin;

// n bytes from host memory src to device memory dst, queued on s through the arena
void h2d(void *dst, const void *src, size_t n, hipStream_t s, const char *what)
{
    if (n == 0)
        return;
    void *st = g_pin.take(n);
    memcpy(st, src, n);
    hipck(hipMemcpyAsync(dst, st, n, hipMemcpyHostToDevice, s), what);
}

// n bytes from device memory src into host memory dst, through the arena;
// waits for s
void d2h_sync(void *dst, const void *src, size_t n, hipStream_t s, const char *what)
{
    if (n == 0)
        return;
    void *st = g_pin.take(n);
    hipck(hipMemcpyAsync(st, src, n, hipMemcpyDeviceToHost, s), what);
    hipck(hipStreamSynchronize(s), "sync");
    memcpy(dst, st, n);
}

// The columns j >= 1 whose seed term at m expands by eq. (4.1): those with
// p_{c+j}^3 <= m, pi(icbrt m) - c of them (icbrt m <= 2^16 for m <= 2^48).
uint32_t seed_rec_cols(uint64_t m, uint32_t c, uint32_t nb)
{
    const uint64_t v = pc_icbrt(m);
    const Tables &T = g_T;
    if (v > T.pi_host_max)
        fail(PC_EINTERNAL, "seed columns beyond the host copy of the pi table");
    const uint64_t pv = v >= 2 ? pc_pi_lookup(T.pi_host, v) : 0;
    return (uint32_t)std::min<uint64_t>(nb, pv > c ? pv - c : 0);
}

struct QueryBufs {
    DevBuf Ub, Xb, Xd, Xbh, e_start, e_count, e_off, e_scount, e_bk, e_boff, e_tmp, e_total, e_clu,
        part, part3, sums, fin, qdev;
    DevBuf work, hot, bounds, tiles_a, trace;
    DevBuf tiles, cnt, wgt, carry_rows, carry_a, carry_b, status, ticket, part_tile_h,
        part_tile_p, part_scan_h, part_scan_p, err;
    DevBuf row_off, blkoff, cntP, wP, carryP, seed_term;
};
QueryBufs g_Q;

hipEvent_t g_fork = nullptr, g_join = nullptr, g_join3 = nullptr;

void init_stream()
{
    if (!g_stream)
        hipck(hipStreamCreateWithFlags(&g_stream, hipStreamNonBlocking), "hipStreamCreate");
    if (!g_stream2)
        hipck(hipStreamCreateWithFlags(&g_stream2, hipStreamNonBlocking), "hipStreamCreate");
    if (!g_stream3)
        hipck(hipStreamCreateWithFlags(&g_stream3, hipStreamNonBlocking), "hipStreamCreate");
    if (!g_join3)
        hipck(hipEventCreateWithFlags(&g_join3, hipEventDisableTiming), "hipEventCreate");
    if (!g_fork)
        hipck(hipEventCreateWithFlags(&g_fork, hipEventDisableTiming), "hipEventCreate");
    if (!g_join)
        hipck(hipEventCreateWithFlags(&g_join, hipEventDisableTiming), "hipEventCreate");
}

// pi at a few points, read back to the host (planning only).
std::vector<uint64_t> lookup(const std::vector<uint64_t> &pts)
{
    Tables &T = g_T;
    size_t n = pts.size();
    ensure(T.lk_in, n * 8, "lookup");
    ensure(T.lk_out, n * 8, "lookup");
    hipck(hipMemcpyAsync(T.lk_in.p, pts.data(), n * 8, hipMemcpyHostToDevice, g_stream), "H2D");
    hipck(pc_launch_lookup(ptr<uint2>(T.pitab), ptr<uint64_t>(T.lk_in), (uint32_t)n,
                           ptr<uint64_t>(T.lk_out), g_stream),
          "lookup");
    std::vector<uint64_t> out(n);
    hipck(hipMemcpyAsync(out.data(), T.lk_out.p, n * 8, hipMemcpyDeviceToHost, g_stream), "D2H");
    hipck(hipStreamSynchronize(g_stream), "sync");
    return out;
}

// Rosser-Schoenfeld: pi(n) < 1.25506 n / ln n for n > 1.
uint64_t pi_upper(uint64_t n)
{
    if (n < 100)
        return 30;
    return (uint64_t)(1.25506 * (double)n / std::log((double)n)) + 64;
}

void ensure_pi(uint64_t need)
{
    Tables &T = g_T;
    if (!T.base_ok) {
        ensure(T.base, 32768 * 4, "base primes"); // the primes below 2^18
        ensure(T.nbase_d, 8, "base count");
        hipck(pc_launch_base_primes(ptr<uint32_t>(T.base), ptr<uint32_t>(T.nbase_d), g_stream),
              "base primes");
        hipck(hipMemcpyAsync(&T.nbase, T.nbase_d.p, 4, hipMemcpyDeviceToHost, g_stream), "D2H");
        hipck(hipStreamSynchronize(g_stream), "sync");
        T.base_ok = true;
    }
    if (T.pi_limit >= need)
        return;
    // up to 2^32 the table doubles as it grows; above, it is sized to the
    // request (isqrt x <= 2^36 for x <= 2^72), the primes above 2^32 held as
    // 64-bit values; the base primes below 2^18 sieve every n < 262147^2
    constexpr uint64_t kPiMax = (1ull << 36) + (1ull << 20), k2_32 = 0xFFFFFFFFull;
    if (need > kPiMax)
        fail(PC_ERANGE, "pi table beyond 2^36 + 2^20 requested");
    uint64_t lim = std::max<uint64_t>({need, std::min(2 * T.pi_limit, k2_32), 1ull << 22});
    uint64_t nent = lim / 64 + 1;
    uint64_t covered = 64 * nent - 1;
    if (covered > k2_32 && need <= k2_32) { // stay within 2^32 when that covers the request
        nent = 1ull << 26;
        covered = k2_32;
    }
    ensure(T.pitab, nent * 8, "pi table");
    ensure(T.cnt_tmp, nent * 4, "pi counts");
    ensure(T.scan_tmp, (nent / 4096 + 2) * 4, "scan");
    ensure(T.primes, (pi_upper(std::min(covered, k2_32)) + 4) * 4, "primes");
    // pi(2^32) = 203280221, so the first prime above 2^32 is p_203280222
    constexpr uint64_t kK32 = 203280222ull;
    if (covered > k2_32)
        ensure(T.primes_hi, (pi_upper(covered) + 4 - kK32) * 8, "primes above 2^32");
    else
        dfree(T.primes_hi);
    hipck(pc_launch_pitab(nent, ptr<uint32_t>(T.base), T.nbase, nullptr, ptr<uint32_t>(T.cnt_tmp),
                          ptr<uint2>(T.pitab), ptr<uint32_t>(T.primes),
                          covered > k2_32 ? ptr<uint64_t>(T.primes_hi) : nullptr,
                          ptr<uint32_t>(T.scan_tmp), g_stream),
          "pi table");
    if (T.cnt_tmp.cap > (1ull << 30)) // up to 2^32 (256 MiB) kept for the next build
        dfree(T.cnt_tmp);
    T.pi_limit = covered;
    T.nprimes = lookup({covered})[0];
    T.k32 = covered > k2_32 ? kK32 : ~0ull;
    if (covered > k2_32 && lookup({k2_32})[0] + 1 != kK32)
        fail(PC_EINTERNAL, "pi(2^32) of the device table is not 203280221");
    T.recip_n = 0; // the primes array was rebuilt
    // the host copy answers the staircase's pi(isqrt(x / lo)): below 2^24 for
    // x < 2^64, at most 2^28 for the queries up to 2^72 (tables above 2^32)
    const uint64_t nh =
        std::min<uint64_t>(nent, (covered > k2_32 ? (1ull << 28) + 64 : 1ull << 24) / 64 + 1);
    if (T.pi_host_cap < nh) {
        if (T.pi_host)
            (void)hipHostFree(T.pi_host);
        T.pi_host = nullptr;
        T.pi_host_cap = 0;
        if (hipHostMalloc((void **)&T.pi_host, nh * 8, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            T.pi_host = nullptr;
            fail(PC_ENOMEM, "pinned host copy of the pi table");
        }
        T.pi_host_cap = nh;
    }
    hipck(hipMemcpyAsync(T.pi_host, T.pitab.p, nh * 8, hipMemcpyDeviceToHost, g_stream),
          "D2H");
    hipck(hipStreamSynchronize(g_stream), "sync");
    T.pi_host_max = 64 * nh - 1;
}

// Row lengths of the count staircase of a query (x, c, nb): a hard leaf of
// p_b has u < x / p_b^2, so the row whose first integer is lo > 0 keeps the
// columns of the primes p_b <= isqrt(x / lo); the first row keeps all nb.
uint32_t row_len(pc_u128 x, uint32_t c, uint32_t nb, uint64_t lo)
{
    if (lo == 0)
        return nb;
    pc_u128 q;
    if ((x >> 64) == 0) {
        q = (uint64_t)x / lo; // (a 64-bit division: the planner takes one per row)
    } else {
        q = x / lo;
        if (q >> 64)
            fail(PC_EINTERNAL, "row length: x / lo beyond 2^64");
    }
    const uint64_t v = pc_isqrt((uint64_t)q);
    const Tables &T = g_T;
    if (v > T.pi_host_max)
        fail(PC_EINTERNAL, "row length beyond the host copy of the pi table");
    const uint64_t pv = pc_pi_lookup(T.pi_host, v);
    return (uint32_t)std::min<uint64_t>(nb, pv > c ? pv - c : 0);
}

void ensure_recip(uint64_t kmax)
{
    Tables &T = g_T;
    if (T.recip_n >= kmax)
        return;
    // (the reciprocal tables cover primes below 2^32 only: p_a+1 < 2^31 for every y)
    uint64_t k = std::min<uint64_t>(std::min(T.nprimes, T.k32 - 1),
                                    std::max<uint64_t>(kmax, 2 * T.recip_n));
    ensure(T.recip, (k + 1) * 8, "reciprocals");
    ensure(T.rcpd, (k + 1) * 8, "reciprocals");
    hipck(pc_launch_recip(ptr<uint32_t>(T.primes), ptr<uint64_t>(T.recip), ptr<double>(T.rcpd),
                          (uint32_t)k, g_stream),
          "reciprocals");
    T.recip_n = k;
}

// The number of squarefree n <= Y, Q(Y) = sum_{d <= isqrt Y} mu(d) floor(Y / d^2)
// (inclusion-exclusion over the squares), for checking the device mu*lpf table.
uint64_t squarefree_count(uint64_t Y)
{
    const uint64_t r = pc_isqrt(Y);
    std::vector<int8_t> mu(r + 1, 1);
    std::vector<uint8_t> comp(r + 1, 0);
    for (uint64_t p = 2; p <= r; p++) {
        if (comp[p])
            continue;
        for (uint64_t k = p; k <= r; k += p) {
            if (k > p)
                comp[k] = 1;
            mu[k] = (int8_t)-mu[k];
        }
        for (uint64_t k = p * p; k <= r; k += p * p)
            mu[k] = 0;
    }
    int64_t q = 0;
    for (uint64_t d = 1; d <= r; d++)
        q += mu[d] * (int64_t)(Y / (d * d));
    return (uint64_t)q;
}

void ensure_mulpf(uint64_t y)
{
    Tables &T = g_T;
    if (T.y_limit >= y)
        return;
    uint64_t Y = std::max<uint64_t>({y, 2 * T.y_limit, 1ull << 20});
    if (Y >= (1ull << 31) - 1)
        Y = (1ull << 31) - 2;
    if (y > Y)
        fail(PC_ERANGE, "y beyond 2^31 - 2");
    ensure_pi(Y);
    uint64_t nsmall = lookup({pc_isqrt(Y)})[0];
    ensure(T.mulpf, (Y + 1) * 4, "mu*lpf table");
    hipck(pc_launch_mulpf(ptr<uint32_t>(T.primes), (uint32_t)nsmall, Y, ptr<int32_t>(T.mulpf),
                          g_stream),
          "mu*lpf table");
    // the table must mark exactly Q(Y) integers squarefree
    ensure(T.chk, 8, "table check");
    hipck(pc_launch_fill_u64(ptr<uint64_t>(T.chk), 1, 0, g_stream), "fill");
    hipck(pc_launch_count_nonzero(ptr<int32_t>(T.mulpf), Y, ptr<unsigned long long>(T.chk),
                                  g_stream),
          "table check");
    uint64_t nsq = 0;
    hipck(hipMemcpyAsync(&nsq, T.chk.p, 8, hipMemcpyDeviceToHost, g_stream), "D2H");
    hipck(hipStreamSynchronize(g_stream), "sync");
    if (nsq != squarefree_count(Y)) {
        dfree(T.mulpf);
        T.y_limit = 0; // rebuilt by the next call that needs it
        fail(PC_EINTERNAL, "mu*lpf table: " + std::to_string(nsq) + " squarefree entries up to " +
                               std::to_string(Y) + ", expected " +
                               std::to_string(squarefree_count(Y)));
    }
    T.y_limit = Y;
}

void ensure_wheel(uint32_t c)
{
    Tables &T = g_T;
    if (T.wheel_ok[c])
        return;
    uint32_t period = 1, Q = 1, phiQ = 1;
    for (uint32_t i = 1; i <= c; i++) {
        Q *= kFirstPrimes[i];
        phiQ *= kFirstPrimes[i] - 1;
        if (i >= 2)
            period *= kFirstPrimes[i];
    }
    uint32_t words = (period + 64) / 32 + 2;
    ensure(T.pattern[c], words * 4, "wheel pattern");
    ensure(T.phitab[c], (size_t)Q * 4, "wheel phi table");
    ensure(T.wres[c], (size_t)phiQ * 4, "wheel residues");
    hipck(pc_launch_wheel(c, ptr<uint32_t>(T.primes), ptr<uint32_t>(T.pattern[c]), words,
                          ptr<uint32_t>(T.phitab[c]), ptr<uint32_t>(T.wres[c]), g_stream),
          "wheel");
    T.pattern_bits[c] = period;
    T.Qc[c] = Q;
    T.phiQ[c] = phiQ;
    T.wheel_ok[c] = true;
}

pc_tables tables_view(uint32_t c)
{
    Tables &T = g_T;
    pc_tables v{};
    v.primes = ptr<uint32_t>(T.primes);
    v.primes_hi = ptr<uint64_t>(T.primes_hi);
    v.k32 = T.k32;
    v.recip = ptr<uint64_t>(T.recip);
    v.rcpd = ptr<double>(T.rcpd);
    v.pitab = ptr<uint2>(T.pitab);
    v.mulpf = ptr<int32_t>(T.mulpf);
    v.pattern = ptr<uint32_t>(T.pattern[c]);
    v.phitab = ptr<uint32_t>(T.phitab[c]);
    v.wres = ptr<uint32_t>(T.wres[c]);
    v.pattern_bits = T.pattern_bits[c];
    v.Qc = T.Qc[c];
    v.phiQ = T.phiQ[c];
    v.rphiQ = 1.0f / (float)T.phiQ[c];
    return v;
}

// Marks every table unbuilt, so that the next call that needs one builds it
// again.  release: also free their memory; else the next build writes into
// the same allocations (after every kernel queued earlier, which may still
// read them, has finished).
void drop_tables(bool release)
{
    Tables &T = g_T;
    if (release) {
        DevBuf *all[] = {&T.base, &T.nbase_d, &T.pitab, &T.primes, &T.primes_hi, &T.cnt_tmp,
                         &T.scan_tmp, &T.recip,
                         &T.rcpd, &T.mulpf, &T.lk_in, &T.lk_out, &T.chk};
        for (DevBuf *b : all)
            dfree(*b);
        for (int c = 0; c <= kWheelC; c++) {
            dfree(T.pattern[c]);
            dfree(T.phitab[c]);
            dfree(T.wres[c]);
        }
        if (T.pi_host)
            (void)hipHostFree(T.pi_host);
        T.pi_host = nullptr;
        T.pi_host_cap = 0;
    } else {
        async_wait_all();
        if (g_stream2)
            (void)hipStreamSynchronize(g_stream2);
        if (g_stream3)
            (void)hipStreamSynchronize(g_stream3);
        if (g_stream)
            (void)hipStreamSynchronize(g_stream);
    }
    for (int c = 0; c <= kWheelC; c++)
        T.wheel_ok[c] = false;
    T.base_ok = false;
    T.pi_limit = T.nprimes = T.recip_n = T.y_limit = 0;
    T.k32 = ~0ull;
    T.pi_host_max = 0;
}

void drop_query_bufs()
{
    QueryBufs &B = g_Q;
    DevBuf *all[] = {&B.Ub, &B.work, &B.hot, &B.bounds, &B.tiles_a, &B.trace, &B.Xb, &B.Xd, &B.Xbh, &B.e_start, &B.e_count, &B.e_off, &B.e_scount, &B.e_bk, &B.e_boff, &B.e_tmp, &B.e_total, &B.e_clu, &B.part, &B.part3,
                     &B.sums, &B.fin, &B.tiles, &B.cnt, &B.wgt, &B.carry_rows,
                     &B.carry_a, &B.carry_b, &B.status, &B.ticket, &B.part_tile_h,
                     &B.part_tile_p, &B.part_scan_h, &B.part_scan_p, &B.err, &B.qdev,
                     &B.row_off, &B.blkoff, &B.cntP, &B.wP, &B.carryP, &B.seed_term};
    for (DevBuf *b : all)
        dfree(*b);
}

pc_i128 to_abi(pc_s128 v)
{
    pc_i128 r;
    r.lo = (uint64_t)v;
    r.hi = (int64_t)(v >> 64);
    return r;
}

// The tuning table's entry for x (pc_alpha_table.h): the one nearest in
// log10 x.  alpha only moves work between the sieve (falls as 1/alpha) and
// the easy leaves (rise), the segment and workgroup shape only how the sieve
// runs; neither ever changes a result.
const pc_alpha_entry &tuned_entry(pc_u128 x)
{
    const double lx = std::log10((double)x);
    const size_t n = sizeof kAlphaTable / sizeof kAlphaTable[0];
    size_t best = 0;
    for (size_t i = 1; i < n; i++)
        if (std::fabs(kAlphaTable[i].log10x - lx) < std::fabs(kAlphaTable[best].log10x - lx))
            best = i;
    return kAlphaTable[best];
}

double default_alpha(pc_u128 x) { return tuned_entry(x).alpha; }

// alpha for a query in a batch round: the least total work rather than the
// least latency of the query alone
double default_batch_alpha(uint64_t x) { return tuned_entry(x).batch_alpha; }

// Integer square and cube roots of a 128-bit x (the host planner of queries
// above 2^64).
uint64_t isqrt128(pc_u128 n)
{
    uint64_t r = (uint64_t)std::sqrt((long double)n);
    while (r > 0 && (pc_u128)r * r > n)
        r--;
    while ((pc_u128)(r + 1) * (r + 1) <= n)
        r++;
    return r;
}

uint64_t icbrt128(pc_u128 n)
{
    uint64_t r = (uint64_t)std::cbrt((long double)n);
    while (r > 0 && (pc_u128)r * r * r > n)
        r--;
    while ((pc_u128)(r + 1) * (r + 1) * (r + 1) <= n)
        r++;
    return r;
}

uint64_t choose_y(pc_u128 x, double alpha)
{
    uint64_t r = icbrt128(x), s = isqrt128(x);
    double yd = std::floor(alpha * (double)r);
    uint64_t y = yd >= (double)s ? s : (uint64_t)yd;
    if (y < r)
        y = r;
    if (y > s)
        y = s;
    return y;
}

struct Knobs {
    uint32_t seg_log2 = 18;
    uint32_t wg = 512;
    bool two_pass = false;
    bool batch = true;
    bool seeded = false;             // windows seeded on their own (Section 4), run last to first
    uint64_t carry_budget = 6ull << 30;
    uint64_t tile_leaves = 1u << 22; // hard-leaf items per tile; 0 = no column splitting
    uint32_t hot_log2 = 15;          // small one-wavefront segments below hot_span * y
    uint32_t hot_wg = 64;
    uint64_t hot_span = 0;           // 0 = no small segments (the measured best at every size)
    bool shape_set = false;          // segment and workgroup named by the caller, not the table
};

Knobs knobs_from(const pc_config *cfg)
{
    Knobs k;
    if (!cfg)
        return k;
    k.shape_set = cfg->segment_kib != 0 || cfg->wg_size != 0;
    switch (cfg->segment_kib) {
    case 0:
        break;
    case 32:
        k.seg_log2 = 18;
        break;
    case 64:
        k.seg_log2 = 19;
        break;
    default:
        fail(PC_EINVAL, "segment_kib must be 32 or 64");
    }
    switch (cfg->wg_size) {
    case 0:
        break;
    case 256:
    case 512:
    case 1024:
        k.wg = cfg->wg_size;
        break;
    default:
        fail(PC_EINVAL, "wg_size must be 256, 512 or 1024");
    }
    // supported (segment, workgroup) shapes: each thread counts one or two whole
    // 512-bit blocks, and the LDS image must fit in 160 KiB
    const bool ok = (k.seg_log2 == 18 && (k.wg == 256 || k.wg == 512)) ||
                    (k.seg_log2 == 19 && (k.wg == 512 || k.wg == 1024));
    if (!ok)
        fail(PC_EINVAL, "unsupported segment_kib / wg_size pair (32: 256|512, 64: 512|1024)");
    k.two_pass = (cfg->flags & PC_FLAG_TWO_PASS) != 0;
    k.batch = (cfg->flags & PC_FLAG_NO_BATCH_LARGE) == 0;
    k.seeded = (cfg->flags & PC_FLAG_SEEDED) != 0;
    if (cfg->carry_budget)
        k.carry_budget = cfg->carry_budget;
    if (cfg->tile_leaves == 0xFFFFFFFFu)
        k.tile_leaves = 0;
    else if (cfg->tile_leaves)
        k.tile_leaves = cfg->tile_leaves;
    if (cfg->small_span)
        k.hot_span = cfg->small_span;
    switch (cfg->small_kib) {
    case 0:
        break;
    case 4:
        k.hot_log2 = 15;
        k.hot_wg = 64;
        break;
    case 8:
        k.hot_log2 = 16;
        k.hot_wg = 64;
        break;
    default:
        fail(PC_EINVAL, "small_kib must be 4 or 8");
    }
    if (cfg->flags & PC_FLAG_NO_SMALL_SEGMENTS)
        k.hot_span = 0;
    return k;
}

// Kernel timing with HIP events recorded on the library stream.
struct EvPair {
    hipEvent_t a = nullptr, b = nullptr;
};
std::vector<EvPair> g_ev;
size_t g_ev_used = 0;

EvPair &ev_next()
{
    if (g_ev_used == g_ev.size()) {
        EvPair e;
        hipck(hipEventCreate(&e.a), "hipEventCreate");
        hipck(hipEventCreate(&e.b), "hipEventCreate");
        g_ev.push_back(e);
    }
    return g_ev[g_ev_used++];
}

// time the launches made by f on stream st; returns the event pair index
template <typename F> size_t timed(F &&f, hipStream_t st = nullptr)
{
    if (!st)
        st = g_stream;
    EvPair &e = ev_next();
    hipck(hipEventRecord(e.a, st), "hipEventRecord");
    f();
    hipck(hipEventRecord(e.b, st), "hipEventRecord");
    return g_ev_used - 1;
}

double ev_ms(size_t i)
{
    float ms = 0;
    hipck(hipEventElapsedTime(&ms, g_ev[i].a, g_ev[i].b), "hipEventElapsedTime");
    return ms;
}

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0)
{
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// Tiles of the window [s0, s0 + rows): segments below plan_end whose estimated
// hard-leaf work exceeds the target are cut into column ranges of about equal
// work (these go first, heaviest first); every other segment is one tile.
void plan_tiles(const pc_tables &T, const pc_query &Q, const Knobs &K, uint32_t log2s,
                uint64_t lo_base, uint64_t seg_base, uint64_t s0, uint64_t rows, uint64_t plan_end,
                std::vector<pc_tile> &tiles)
{
    QueryBufs &B = g_Q;
    tiles.clear();
    std::vector<uint8_t> split(rows, 0);
    if (K.tile_leaves && plan_end > s0) {
        const uint64_t np = plan_end - s0;
        ensure(B.work, np * 8, "tile plan");
        hipck(pc_launch_seg_work(T, Q, log2s, lo_base, seg_base, s0, (uint32_t)np,
                                 ptr<uint64_t>(B.work), g_stream),
              "tile plan");
        std::vector<uint64_t> work(np);
        d2h_sync(work.data(), B.work.p, np * 8, g_stream, "D2H");
        // The target: K.tile_leaves, or less when the whole window holds little
        // leaf work, so that no tile outlasts the rest of the launch (about
        // 768 workgroups run at once; a tile should carry at most twice its
        // share of the estimated work).
        uint64_t total = 0;
        for (uint64_t i = 0; i < np; i++)
            total += work[i];
        const uint64_t target =
            std::clamp<uint64_t>(total / 384, std::min<uint64_t>(1u << 16, K.tile_leaves),
                                 K.tile_leaves);
        std::vector<uint4> hot;
        uint32_t off = 0;
        for (uint64_t i = 0; i < np; i++)
            if (work[i] > target) {
                uint64_t k = (work[i] + target - 1) / target;
                k = std::min<uint64_t>(k, std::min<uint64_t>(4096, Q.nb));
                if (k < 2)
                    continue;
                hot.push_back(uint4{(uint32_t)(s0 + i), (uint32_t)k, off, 0});
                off += (uint32_t)k + 1;
            }
        if (!hot.empty()) {
            std::sort(hot.begin(), hot.end(), [&](const uint4 &a, const uint4 &b) {
                return work[a.x - s0] > work[b.x - s0];
            });
            off = 0;
            for (uint4 &h : hot) {
                h.z = off;
                off += h.y + 1;
            }
            ensure(B.hot, hot.size() * sizeof(uint4), "tile plan");
            ensure(B.bounds, (size_t)off * 4, "tile plan");
            h2d(B.hot.p, hot.data(), hot.size() * sizeof(uint4), g_stream, "H2D");
            hipck(pc_launch_seg_split(T, Q, log2s, lo_base, seg_base, ptr<uint4>(B.hot),
                                      (uint32_t)hot.size(), ptr<uint32_t>(B.bounds), g_stream),
                  "tile split");
            std::vector<uint32_t> bd(off);
            d2h_sync(bd.data(), B.bounds.p, (size_t)off * 4, g_stream, "D2H");
            for (const uint4 &h : hot) {
                const uint32_t *b = bd.data() + h.z;
                for (uint32_t j = 0; j < h.y; j++)
                    if (b[j] < b[j + 1])
                        tiles.push_back(pc_tile{h.x, b[j], b[j + 1], 0});
                split[h.x - s0] = 1;
            }
        }
    }
    for (uint64_t r = 0; r < rows; r++)
        if (!split[r])
            tiles.push_back(pc_tile{(uint32_t)(s0 + r), 0, Q.ncol, 0});
}

// Full decomposition for one (x, y); x >= 8, icbrt(x) <= y <= isqrt(x),
// x <= 2^72 (above 2^64 X_b, S1's quotients and pi(x) itself may take 128
// bits; the sieve's and the leaves' quotients all stay below 2^64).
constexpr pc_u128 kWideMax = (pc_u128)1 << 72;

void run_query(pc_u128 x, uint64_t y, const Knobs &K, pc_result *res)
{
    auto t0 = clk::now();
    init_stream();
    // the plan copies of an earlier query (one that failed part way too) are done
    hipck(hipStreamSynchronize(g_stream), "sync");
    g_pin.reset();
    QueryBufs &B = g_Q;
    const uint64_t x_hi = (uint64_t)(x >> 64);
    if (x > kWideMax)
        fail(PC_ERANGE, "x beyond 2^72");
    const uint64_t sx = isqrt128(x);
    if ((x / y) >> 64)
        fail(PC_ERANGE, "x / y beyond 2^64");
    const uint64_t z = (uint64_t)(x / y);
    ensure_pi(std::max<uint64_t>({sx, y, 1024}) + 1);
    std::vector<uint64_t> lk = lookup({y, sx, pc_isqrt(z)});
    const uint64_t a = lk[0], kx = lk[1], bmax = lk[2];
    const uint32_t c = (uint32_t)std::min<uint64_t>(kWheelC, a);
    if (c < 1)
        fail(PC_EINVAL, "y too small");
    if (x_hi && c != 6)
        fail(PC_EINTERNAL, "queries above 2^64 need the wheel of the primes up to 13");
    ensure_mulpf(y);
    ensure_recip(a + 1);
    ensure_wheel(c);
    hipck(hipStreamSynchronize(g_stream), "sync");
    const double ms_tables = ms_since(t0);

    const pc_tables T = tables_view(c);
    pc_query Q{};
    Q.x = (uint64_t)x;
    Q.x_hi = x_hi;
    Q.xd = (double)x;
    Q.y = y;
    Q.z = z;
    Q.y1 = y + 1;
    Q.recip_y1 = pc_recip(y + 1);
    Q.sqrtx = sx;
    Q.sqrty = pc_isqrt(y);
    Q.Qc = T.Qc;
    Q.recip_Qc = pc_recip(T.Qc);
    Q.c = c;
    Q.a = (uint32_t)a;
    Q.bmax = (uint32_t)bmax;
    Q.nb = bmax > c ? (uint32_t)(bmax - c) : 0;
    Q.ncol = Q.nb + 1;
    Q.kx = (uint32_t)kx;

    // Rows of the sieve: nA one-wavefront segments of 2*SA integers covering
    // the leaf-dense low end up to about hot_span * y, then nB workgroup
    // segments of 2*S integers, together covering [0, z].
    const uint64_t S = 1ull << K.seg_log2, SA = 1ull << K.hot_log2;
    uint64_t nA = 0;
    if (K.hot_span) {
        const uint64_t uA = std::min<uint64_t>(z + 1, K.hot_span * y);
        nA = (uA + 2 * SA - 1) / (2 * SA);
    }
    const uint64_t baseB = nA * 2 * SA;
    const uint64_t nB = baseB > z ? 0 : (z - baseB) / (2 * S) + 1;
    const uint64_t nseg = nA + nB;
    Q.sieve_end = baseB + nB * 2 * S;
    Q.nseg = nseg;
    g_ev_used = 0;

    // --- per-query tables and the leaves outside the sieve ---
    ensure(B.Xb, (a + 2) * 8, "X_b");
    ensure(B.Xd, (a + 2) * 8, "X_b");
    Q.Xb = Q.Xb_w = ptr<uint64_t>(B.Xb);
    Q.Xd = ptr<double>(B.Xd);
    Q.Xbh = nullptr;
    if (x_hi) {
        ensure(B.Xbh, (a + 2) * 4, "X_b");
        Q.Xbh = ptr<uint32_t>(B.Xbh);
    }
    hipck(pc_launch_xb(T, Q, g_stream), "X_b");

    ensure(B.sums, sizeof(pc_sums), "sums");
    ensure(B.fin, sizeof(pc_final), "final");
    ensure(B.e_total, 32, "easy total");
    hipck(pc_launch_fill_u64(ptr<uint64_t>(B.sums), sizeof(pc_sums) / 8, 0, g_stream), "fill");
    pc_sums *sums = ptr<pc_sums>(B.sums);
    Q.sums = sums;

    const uint32_t s1_blocks = (uint32_t)std::min<uint64_t>(2048, y / 256 + 1);
    const uint32_t ls_blocks = (uint32_t)(a / 256 + 1);
    const uint32_t ez_blocks = 4096;
    ensure(B.part, (size_t)std::max<uint32_t>({s1_blocks, ls_blocks, ez_blocks}) * 16, "partials");
    ensure(B.part3, (size_t)ez_blocks * 16, "partials");
    auto t1 = clk::now();
    const size_t ev_s1 = timed(
        [&] { hipck(pc_launch_s1(T, Q, ptr<pc_s128>(B.part), s1_blocks, g_stream), "S1"); });
    hipck(pc_launch_sum128(ptr<pc_s128>(B.part), s1_blocks, &sums->s1, g_stream), "S1 sum");

    ensure(B.e_start, (a + 2) * 8, "easy ranges");
    ensure(B.e_count, (a + 2) * 8, "easy ranges");
    ensure(B.e_off, (a + 2) * 8, "easy offsets");
    ensure(B.e_scount, (a + 2) * 8, "easy ranges");
    const uint64_t nband = a / PC_EZ_BAND + 1;
    ensure(B.e_bk, 2 * nband * 4, "easy bands");
    ensure(B.e_boff, 2 * nband * 8, "easy bands");

    ensure(B.e_clu, (a + 2) * 16, "easy clusters");
    ensure(B.e_tmp, ((a + 2) / 4096 + 2) * 8, "scan");
    ensure(B.Ub, (a + 2) * 16, "hard-leaf u ranges");
    Q.Ub = Q.Ub_w = ptr<ulonglong2>(B.Ub);
    Q.e_start = ptr<uint64_t>(B.e_start);
    Q.e_count = ptr<uint64_t>(B.e_count);
    Q.e_off = ptr<uint64_t>(B.e_off);
    Q.e_scount = ptr<uint64_t>(B.e_scount);
    Q.e_bk = ptr<uint32_t>(B.e_bk);
    Q.e_boff = ptr<uint64_t>(B.e_boff);
    Q.e_total = ptr<uint64_t>(B.e_total);
    Q.e_clu = ptr<uint4>(B.e_clu);
    hipck(pc_launch_leaf_setup(T, Q, ptr<pc_s128>(B.part), ls_blocks, g_stream), "leaf setup");
    hipck(pc_launch_sum128(ptr<pc_s128>(B.part), ls_blocks, &sums->s2t, g_stream), "S2t sum");
    hipck(pc_launch_strip(ptr<uint64_t>(B.e_count), ptr<uint64_t>(B.e_off), a + 1, g_stream),
          "strip");
    hipck(pc_launch_scan_u64(ptr<uint64_t>(B.e_off), a + 1, ptr<uint64_t>(B.e_tmp),
                             ptr<uint64_t>(B.e_total), g_stream),
          "easy scan");
    hipck(pc_launch_easy_bands(T, Q, g_stream), "easy bands");
    for (int kind = 0; kind < 2; kind++)
        hipck(pc_launch_scan_u64(ptr<uint64_t>(B.e_boff) + kind * nband, nband,
                                 ptr<uint64_t>(B.e_tmp), ptr<uint64_t>(B.e_total) + 1 + kind,
                                 g_stream),
              "easy scan");
    // The easy leaves touch nothing the sieve writes: they run on the second
    // stream once the last sieve window is queued, and rejoin before the
    // combination.  Both kernels keep every CU busy, so running them side by
    // side gains nothing (measured); after the windows, neither delays the
    // other's launches.
    size_t ev_easy = 0;
    bool forked = false;
    auto fork_easy = [&]() {
        if (forked)
            return;
        forked = true;
        hipck(hipEventRecord(g_fork, g_stream), "hipEventRecord");
        hipck(hipStreamWaitEvent(g_stream2, g_fork, 0), "hipStreamWaitEvent");
        // the bands (integer issue) and the candidates (table reads) side by
        // side on two streams, each with its own partials
        ev_easy = timed(
            [&] {
                hipck(hipStreamWaitEvent(g_stream3, g_fork, 0), "hipStreamWaitEvent");
                hipck(pc_launch_easy(T, Q, ptr<pc_s128>(B.part3), ez_blocks, g_stream3), "easy");
                hipck(hipEventRecord(g_join3, g_stream3), "hipEventRecord");
                hipck(pc_launch_easy_band(T, Q, ptr<pc_s128>(B.part), ez_blocks, g_stream2),
                      "easy");
                hipck(hipStreamWaitEvent(g_stream2, g_join3, 0), "hipStreamWaitEvent");
            },
            g_stream2);
        hipck(pc_launch_sum128(ptr<pc_s128>(B.part), ez_blocks, &sums->s2e, g_stream2),
              "S2e sum");
        hipck(pc_launch_sum128(ptr<pc_s128>(B.part3), ez_blocks, &sums->s2e, g_stream2),
              "S2e sum");
        hipck(hipEventRecord(g_join, g_stream2), "hipEventRecord");
    };
    (void)t1;

    // --- the sieve of [1, z] in windows of segments ---
    auto t2 = clk::now();
    std::vector<size_t> ev_sieve, ev_scan, ev_seed;
    // Row lengths of the count staircase: a hard leaf of p_b has u < x / p_b^2,
    // so row r (first integer lo_r) stores the columns of the primes
    // p_b <= isqrt(x / lo_r), and the first row stores every column.
    std::vector<uint32_t> rowlen(nseg);
    for (uint64_t r = 0; r < nseg; r++)
        rowlen[r] = row_len(x, c, Q.nb, r < nA ? r * 2 * SA : baseB + (r - nA) * 2 * S);
    // windows of rows within the carry budget (cells of cnt and w, or of cnt
    // and the carries, plus the P2 column's per-row words)
    const uint64_t per_cell = K.two_pass ? 12 : 8, per_row = K.two_pass ? 12 : 8;
    std::vector<uint64_t> win_start{0};
    uint64_t max_rows = 0, max_cells = 0, cells_total = 0;
    {
        uint64_t cells = 0, rows = 0;
        for (uint64_t r = 0; r < nseg; r++) {
            if (rows && (cells + rowlen[r]) * per_cell + (rows + 1) * per_row > K.carry_budget) {
                win_start.push_back(r);
                cells = rows = 0;
            }
            cells += rowlen[r];
            rows++;
            max_rows = std::max(max_rows, rows);
            max_cells = std::max(max_cells, cells);
            cells_total += rowlen[r];
        }
        win_start.push_back(nseg);
    }
    const uint64_t nwin = win_start.size() - 1;
    const uint32_t R = (uint32_t)std::clamp<uint64_t>(max_rows / 256, 16, 1024);
    uint64_t max_chunks = (max_rows + R - 1) / R, max_tickets = 0;
    // the scan's tickets per window: blocks of 256 columns of each chunk's first row
    std::vector<std::vector<uint32_t>> blkoffs(nwin);
    for (uint64_t w = 0; w < nwin; w++) {
        std::vector<uint32_t> &bo = blkoffs[w];
        bo.push_back(0);
        for (uint64_t r = win_start[w]; r < win_start[w + 1]; r += R)
            bo.push_back(bo.back() + (rowlen[r] + 255) / 256);
        max_tickets = std::max<uint64_t>(max_tickets, bo.back());
    }

    ensure(B.cnt, max_cells * 4, "counts");
    if (!K.two_pass)
        ensure(B.wgt, max_cells * 4, "leaf weights");
    else
        ensure(B.carry_rows, max_cells * 8, "carries");
    ensure(B.cntP, max_rows * 4, "P2 counts");
    if (!K.two_pass)
        ensure(B.wP, max_rows * 4, "P2 weights");
    else
        ensure(B.carryP, max_rows * 8, "P2 carries");
    ensure(B.row_off, (max_rows + 1) * 8, "row offsets");
    ensure(B.blkoff, (max_chunks + 1) * 4, "scan blocks");
    ensure(B.carry_a, (size_t)Q.ncol * 8, "carry");
    ensure(B.carry_b, (size_t)Q.ncol * 8, "carry");
    if (K.seeded)
        ensure(B.seed_term, (size_t)Q.ncol * 8, "seed terms");
    ensure(B.status, max_tickets * 256 * 8 + 8, "look-back status");
    ensure(B.ticket, 8, "ticket");
    ensure(B.part_scan_h, max_tickets * 16 + 16, "scan partials");
    ensure(B.part_scan_p, 16, "scan partials");
    ensure(B.err, 8, "error flag");
    hipck(pc_launch_fill_u64(ptr<uint64_t>(B.carry_a), Q.ncol, 0, g_stream), "fill");
    // the query as the sieve reads it: one entry of a device array
    Q.row_off = ptr<uint64_t>(B.row_off);
    Q.cnt = ptr<uint32_t>(B.cnt);
    Q.wgt = ptr<int32_t>(B.wgt);
    Q.carry = ptr<uint64_t>(B.carry_rows);
    Q.cntP = ptr<uint32_t>(B.cntP);
    Q.wP = ptr<int32_t>(B.wP);
    Q.carryP = ptr<uint64_t>(B.carryP);
    ensure(B.qdev, sizeof(pc_query), "query");
    hipck(hipMemcpyAsync(B.qdev.p, &Q, sizeof Q, hipMemcpyHostToDevice, g_stream), "H2D");
    hipck(pc_launch_fill_u64(ptr<uint64_t>(B.err), 1, 0, g_stream), "fill");

    // PICOUNT_TILE_TRACE=<path>: append one line per sieve tile (profiling aid)
    FILE *trace_file = nullptr;
    if (const char *tp = std::getenv("PICOUNT_TILE_TRACE"))
        trace_file = std::fopen(tp, "a");
    std::vector<pc_tile> tiles_a, tiles_b;
    uint64_t ntiles_total = 0;
    uint64_t *cin = ptr<uint64_t>(B.carry_a), *cout = ptr<uint64_t>(B.carry_b);
    const int bflag = K.batch ? 0 : 0x100;
    for (uint64_t wi = 0; wi < nwin; wi++) {
        // seeded windows need nothing from each other: they run last to first
        const uint64_t w = K.seeded ? nwin - 1 - wi : wi;
        const uint64_t r0 = win_start[w], r1 = win_start[w + 1], rows = r1 - r0;
        if (K.seeded && w > 0) {
            // the window's carries on their own: every integer below its first
            // one, phi(lo - 1, c + j) in column j (Section 4)
            const uint64_t lo_w = r0 < nA ? r0 * 2 * SA : baseB + (r0 - nA) * 2 * S;
            const uint32_t nrec = seed_rec_cols(lo_w - 1, c, Q.nb);
            ev_seed.push_back(timed([&] {
                hipck(pc_launch_seed(T, c, lo_w - 1, Q.nb, nrec, g_T.pi_limit,
                                     ptr<int64_t>(B.seed_term), cin, ptr<int32_t>(B.err),
                                     g_stream),
                      "seeds");
            }));
        } else if (K.seeded) {
            hipck(pc_launch_fill_u64(cin, Q.ncol, 0, g_stream), "fill");
        }
        {
            std::vector<uint64_t> off(rows + 1, 0);
            for (uint64_t r = 0; r < rows; r++)
                off[r + 1] = off[r] + rowlen[r0 + r];
            h2d(B.row_off.p, off.data(), off.size() * 8, g_stream, "row offsets");
            h2d(B.blkoff.p, blkoffs[w].data(), blkoffs[w].size() * 4, g_stream, "scan blocks");
        }
        // rows [r0, min(r1, nA)) are small segments, the rest workgroup segments
        tiles_a.clear();
        for (uint64_t r = r0; r < std::min(r1, nA); r++)
            tiles_a.push_back(pc_tile{(uint32_t)r, 0, Q.ncol, 0});
        tiles_b.clear();
        if (r1 > nA) {
            const uint64_t b0 = std::max(r0, nA);
            const uint64_t hot_end = std::max<uint64_t>(64 * y, z / 32);
            const uint64_t plan_end =
                hot_end <= baseB ? b0 : std::min(r1, nA + (hot_end - baseB) / (2 * S) + 1);
            plan_tiles(T, Q, K, K.seg_log2, baseB, nA, b0, r1 - b0, std::max(b0, plan_end),
                       tiles_b);
        }
        ntiles_total += tiles_a.size() + tiles_b.size();
        ensure(B.tiles_a, tiles_a.size() * sizeof(pc_tile), "tiles");
        ensure(B.tiles, tiles_b.size() * sizeof(pc_tile), "tiles");
        const size_t npart = std::max(tiles_a.size(), tiles_b.size());
        ensure(B.part_tile_h, npart * 16, "tile partials");
        ensure(B.part_tile_p, npart * 16, "tile partials");
        h2d(B.tiles_a.p, tiles_a.data(), tiles_a.size() * sizeof(pc_tile), g_stream, "tiles");
        h2d(B.tiles.p, tiles_b.data(), tiles_b.size() * sizeof(pc_tile), g_stream, "tiles");
        auto sieve_args = [&](bool small) {
            pc_sieve_args A{};
            A.T = T;
            A.Qs = ptr<pc_query>(B.qdev);
            A.tiles = ptr<pc_tile>(small ? B.tiles_a : B.tiles);
            A.ntiles = (uint32_t)(small ? tiles_a.size() : tiles_b.size());
            A.seg0 = r0;
            A.lo_base = small ? 0 : baseB;
            A.seg_base = small ? 0 : nA;
            A.part_hard = ptr<pc_s128>(B.part_tile_h);
            A.part_p2 = ptr<pc_s128>(B.part_tile_p);
            A.err = ptr<int32_t>(B.err);
            return A;
        };
        // one sieve launch per geometry; the tile partials are folded right after
        auto sieve = [&](bool small, int mode) {
            pc_sieve_args A = sieve_args(small);
            if (A.ntiles == 0)
                return;
            if (trace_file) {
                ensure(B.trace, (size_t)A.ntiles * PC_TRACE_W * 4, "tile trace");
                hipck(pc_launch_fill_u64(ptr<uint64_t>(B.trace),
                                         (uint64_t)A.ntiles * PC_TRACE_W / 2, 0, g_stream),
                      "fill");
                A.trace = ptr<uint32_t>(B.trace);
            }
            ev_sieve.push_back(timed([&] {
                hipck(pc_launch_sieve(A, small ? K.hot_log2 : K.seg_log2, small ? K.hot_wg : K.wg,
                                      mode | bflag, g_stream),
                      "sieve");
            }));
            if (trace_file) { // per-tile profile: segment, columns, ticks (100 MHz), work
                std::vector<uint32_t> tr((size_t)A.ntiles * PC_TRACE_W);
                hipck(hipMemcpyAsync(tr.data(), B.trace.p, tr.size() * 4,
                                     hipMemcpyDeviceToHost, g_stream),
                      "D2H");
                hipck(hipStreamSynchronize(g_stream), "sync");
                const std::vector<pc_tile> &tl = small ? tiles_a : tiles_b;
                for (uint32_t i = 0; i < A.ntiles; i++) {
                    std::fprintf(trace_file, "%u %u %u %u %d", (unsigned)w, tl[i].seg,
                                 tl[i].col_lo, tl[i].col_hi, small ? 1 : 0);
                    for (uint32_t k = 0; k < PC_TRACE_W; k++)
                        std::fprintf(trace_file, " %u", tr[(size_t)i * PC_TRACE_W + k]);
                    std::fputc('\n', trace_file);
                }
            }
            if (mode != PC_MODE_COUNT) {
                hipck(pc_launch_sum128(ptr<pc_s128>(B.part_tile_h), A.ntiles, &sums->hard_local,
                                       g_stream),
                      "sum");
                hipck(pc_launch_sum128(ptr<pc_s128>(B.part_tile_p), A.ntiles, &sums->p2_local,
                                       g_stream),
                      "sum");
            }
        };
        const int first = K.two_pass ? PC_MODE_COUNT : PC_MODE_TALLY;
        sieve(true, first);
        sieve(false, first);

        pc_scan_args SA{};
        SA.cnt = ptr<uint32_t>(B.cnt);
        SA.wgt = ptr<int32_t>(B.wgt);
        SA.row_off = ptr<uint64_t>(B.row_off);
        SA.blkoff = ptr<uint32_t>(B.blkoff);
        SA.carry_rows = ptr<uint64_t>(B.carry_rows);
        SA.cntP = ptr<uint32_t>(B.cntP);
        SA.wP = ptr<int32_t>(B.wP);
        SA.carryP = ptr<uint64_t>(B.carryP);
        SA.carry_in = cin;
        SA.carry_out = cout;
        SA.status = ptr<uint64_t>(B.status);
        SA.ticket = ptr<uint32_t>(B.ticket);
        SA.part_hard = ptr<pc_s128>(B.part_scan_h);
        SA.part_p2 = ptr<pc_s128>(B.part_scan_p);
        SA.err = ptr<int32_t>(B.err);
        SA.nrows = rows;
        SA.nb = Q.nb;
        SA.rows_per_chunk = R;
        SA.nchunk = (uint32_t)((rows + R - 1) / R);
        SA.nticket = blkoffs[w].back();
        hipck(pc_launch_fill_u64(ptr<uint64_t>(B.status), (uint64_t)SA.nticket * 256, 0,
                                 g_stream),
              "fill");
        hipck(pc_launch_fill_u64(ptr<uint64_t>(B.ticket), 1, 0, g_stream), "fill");
        ev_scan.push_back(timed([&] {
            hipck(pc_launch_scan(SA, K.two_pass ? PC_MODE_COUNT : PC_MODE_TALLY, g_stream),
                  "scan");
        }));
        if (K.two_pass) {
            sieve(true, PC_MODE_LEAVES);
            sieve(false, PC_MODE_LEAVES);
        } else {
            hipck(pc_launch_sum128(ptr<pc_s128>(B.part_scan_h), SA.nticket, &sums->hard_dot,
                                   g_stream),
                  "sum");
            hipck(pc_launch_sum128(ptr<pc_s128>(B.part_scan_p), 1, &sums->p2_dot, g_stream),
                  "sum");
        }
        if (!K.seeded)
            std::swap(cin, cout);
    }
    if (trace_file)
        std::fclose(trace_file);
    fork_easy();
    hipck(hipStreamWaitEvent(g_stream, g_join, 0), "hipStreamWaitEvent");
    hipck(pc_launch_combine(sums, Q, kx, ptr<pc_final>(B.fin), g_stream), "combine");
    pc_final fin{};
    pc_sums hs{};
    int32_t err = 0;
    uint64_t e_items = 0;
    hipck(hipMemcpyAsync(&e_items, B.e_total.p, 8, hipMemcpyDeviceToHost, g_stream), "D2H");
    hipck(hipMemcpyAsync(&hs, B.sums.p, sizeof hs, hipMemcpyDeviceToHost, g_stream), "D2H");
    hipck(hipMemcpyAsync(&fin, B.fin.p, sizeof fin, hipMemcpyDeviceToHost, g_stream), "D2H");
    hipck(hipMemcpyAsync(&err, B.err.p, 4, hipMemcpyDeviceToHost, g_stream), "D2H");
    hipck(hipStreamSynchronize(g_stream), "sync");
    const double ms_sieve = ms_since(t2);
    if (err & 1)
        fail(PC_EINTERNAL, "look-back scan did not complete");
    if (err & 8)
        fail(PC_EINTERNAL, "a sieving column before the cut lay outside its row's stored range");
    if (err & 16)
        fail(PC_EINTERNAL, "window seeds: pi table too short, stack too deep or a negative phi");
    if (err & 32)
        fail(PC_EINTERNAL, "a segment's carried unsieved count disagreed with its recount");
    if (err)
        fail(PC_EINTERNAL, "a leaf or P2 quotient fell outside its segment");
    if (fin.ok == 0 || (fin.ok == 2 && !x_hi))
        fail(PC_EINTERNAL, "pi(x) outside [0, 2^64)");

    if (res) {
        memset(res, 0, sizeof *res);
        res->x = (uint64_t)x;
        res->x_hi = x_hi;
        res->y = y;
        res->a = a;
        res->c = c;
        res->z = z;
        res->bmax = bmax;
        res->pi = fin.pi;
        res->pi_hi = fin.pi_hi;
        res->s1 = to_abi(fin.s1);
        res->s2_trivial = to_abi(fin.s2t);
        res->s2_easy = to_abi(fin.s2e);
        res->s2_hard = to_abi(fin.s2h);
        res->p2 = to_abi(fin.p2);
        res->phi = to_abi(fin.phi);
        res->n_trivial = hs.n_trivial;
        res->n_p2 = kx > a ? kx - a : 0;
        res->n_s1 = hs.n_s1;
        res->n_easy = hs.n_easy;
        res->n_hard = hs.n_hard;
        res->n_easy_items = e_items + hs.n_easy_terms;
        res->crossings = hs.crossings;
        res->segments = nseg;
        res->tiles = ntiles_total;
        res->windows = nwin;
        res->segment_bits = S;
        res->small_segments = nA;
        res->device_bytes = g_dev_peak;
        res->ms_total = ms_since(t0);
        res->ms_tables = ms_tables;
        float ms_lv = 0; // S1 start to the end of the easy leaves (GPU clock)
        hipck(hipEventElapsedTime(&ms_lv, g_ev[ev_s1].a, g_ev[ev_easy].b), "hipEventElapsedTime");
        res->ms_leaves = ms_lv;
        res->ms_sieve = ms_sieve;
        res->ms_k_s1 = ev_ms(ev_s1);
        res->ms_k_easy = ev_ms(ev_easy);
        for (size_t i : ev_sieve)
            res->ms_k_sieve += ev_ms(i);
        for (size_t i : ev_scan)
            res->ms_k_scan += ev_ms(i);
        for (size_t i : ev_seed)
            res->ms_k_seed += ev_ms(i);
        res->sieve_launches = (uint32_t)ev_sieve.size();
        res->scan_launches = (uint32_t)ev_scan.size();
    }
}

uint64_t small_pi(uint64_t x)
{
    init_stream();
    ensure_pi(kSmallX);
    return lookup({x})[0];
}

void check_y(uint64_t x, uint64_t y)
{
    if (x < 8)
        fail(PC_EINVAL, "x must be >= 8");
    if (y < pc_icbrt(x) || y > pc_isqrt(x))
        fail(PC_EINVAL, "y must satisfy icbrt(x) <= y <= isqrt(x)");
}

template <typename F> pc_status guarded(F &&f)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    t_err.clear();
    try {
        f();
        return PC_OK;
    } catch (const pc_error &e) {
        t_err = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        t_err = "host allocation failed";
        return PC_ENOMEM;
    } catch (...) {
        t_err = "unexpected exception";
        return PC_EINTERNAL;
    }
}

void pi_one(pc_u128 x, const Knobs &K, double alpha, pc_result *res, uint64_t *pi)
{
    if (std::isnan(alpha) || alpha < 0)
        fail(PC_EINVAL, "alpha must be >= 0 (0 = tuned)");
    if (x < kSmallX) {
        uint64_t v = small_pi((uint64_t)x);
        if (res) {
            memset(res, 0, sizeof *res);
            res->x = (uint64_t)x;
            res->pi = v;
        }
        *pi = v;
        return;
    }
    if (alpha == 0)
        alpha = default_alpha(x);
    const uint64_t y = choose_y(x, alpha);
    Knobs Kx = K;
    if (!K.shape_set) { // the tuned segment and workgroup for this size
        const pc_alpha_entry &e = tuned_entry(x);
        Kx.seg_log2 = e.seg_kib == 64 ? 19 : 18;
        Kx.wg = e.wg;
    }
    pc_result r;
    run_query(x, y, Kx, &r);
    *pi = r.pi;
    if (res)
        *res = r;
}


// ---------------------------------------------------------------------------
// Batches.  Queries x >= kSmallX go through rounds: each round holds as many
// queries (in order) as fit the carry budget with every row of their sieve
// counts resident, and runs them together: one set-up pass, one easy-leaf
// pass, one sieve launch whose tiles name their query, one carry pass and one
// combination, captured as a HIP graph (PC_FLAG_NO_GRAPH: launched directly).
// A query whose counts alone exceed the budget runs by itself, windowed.
// ---------------------------------------------------------------------------
struct BatchQuery {
    uint64_t x, y, a, kx, bmax, z, nseg;
    uint32_t c, nb, ncol;
    size_t idx; // position in the caller's array
    uint64_t bytes() const { return nseg * ncol * 8; }
};

constexpr uint32_t kBatchLog2S = 18; // 32 KiB segments
constexpr uint32_t kBatchWG = 512;

size_t r256(size_t v) { return (v + 255) & ~(size_t)255; }

// A query's chunk of a round arena: X_b, Ub, four easy arrays, e_clu, Xd, bands,
// counts and weights (cells of the count staircase), the P2 column's counts
// and weights, each rounded up to 256 bytes exactly as round_queries takes
// them.
size_t query_chunk(const BatchQuery &b, uint64_t cells)
{
    const size_t na = b.a + 2;
    const size_t nband = b.a / PC_EZ_BAND + 1;
    return 6 * r256(na * 8) + 2 * r256(na * 16) + r256(2 * nband * 4) + r256(2 * nband * 8) +
           2 * r256(cells * 4) + 2 * r256(b.nseg * 4);
}

// What the host builds for one round: the arena layout (sums, easy totals,
// results, then each query's chunk), the sieve tiles, and the block tables of
// the flat kernels (the query of each block and each query's first block).
struct RoundPlan {
    size_t arena = 0, o_sums = 0, o_et = 0, o_fin = 0;
    std::vector<size_t> o_q;
    std::vector<uint64_t> roff;   // every query's row offsets (nseg + 1 each), uploaded
    std::vector<size_t> o_roff;   // where each query's offsets start in roff
    std::vector<uint64_t> cells;  // stored cells of each query's staircase
    std::vector<pc_tile> tiles;
    std::vector<uint32_t> blk;
    size_t t_xb = 0, t_s1 = 0, t_ez = 0, t_sc = 0;
    uint32_t nb_xb = 0, nb_s1 = 0, nb_ez = 0, nb_sc = 0;
};

// Everything one batch round keeps while it is on the device: its stream
// (null: the library stream), buffers, pinned results, and the host arrays
// its copies read from.
struct BatchSlot {
    hipStream_t st = nullptr;
    DevBuf arena, qs, tiles, blk, roff, err;
    pc_final *h_fin = nullptr; // pinned
    size_t h_fin_cap = 0;
    int32_t *h_err = nullptr;  // pinned
    hipEvent_t done = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<BatchQuery> R;
    std::vector<pc_query> Qv;
    RoundPlan plan;
    uint64_t bytes = 0;
    bool busy = false;
};

// grow a slot buffer, waiting only for the slot's own stream
void slot_ensure(BatchSlot &sl, DevBuf &b, size_t bytes, const char *what)
{
    if (bytes == 0)
        bytes = 16;
    if (b.cap >= bytes)
        return;
    if (b.p) {
        (void)hipStreamSynchronize(sl.st ? sl.st : g_stream);
        (void)hipFree(b.p);
        g_dev_bytes -= b.cap;
        b.p = nullptr;
        b.cap = 0;
    }
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(PC_ENOMEM, std::string("device allocation of ") + std::to_string(bytes) +
                            " bytes for " + what + " failed");
    }
    b.cap = bytes;
    g_dev_bytes += bytes;
    g_dev_peak = std::max<size_t>(g_dev_peak.load(), g_dev_bytes.load());
}

void slot_release(BatchSlot &sl)
{
    if (sl.st)
        (void)hipStreamSynchronize(sl.st);
    for (DevBuf *b : {&sl.arena, &sl.qs, &sl.tiles, &sl.blk, &sl.roff, &sl.err})
        if (b->p) {
            (void)hipFree(b->p);
            g_dev_bytes -= b->cap;
            b->p = nullptr;
            b->cap = 0;
        }
    if (sl.h_fin)
        (void)hipHostFree(sl.h_fin);
    if (sl.h_err)
        (void)hipHostFree(sl.h_err);
    if (sl.done)
        (void)hipEventDestroy(sl.done);
    if (sl.st)
        (void)hipStreamDestroy(sl.st);
    sl = BatchSlot{};
}

// The round's arena layout, block tables and tiles.
void plan_round(const std::vector<BatchQuery> &R, RoundPlan &P)
{
    const uint32_t nq = (uint32_t)R.size();
    P.arena = 0;
    auto take = [&](size_t bytes) {
        const size_t o = P.arena;
        P.arena += r256(bytes);
        return o;
    };
    P.o_sums = take(nq * sizeof(pc_sums));
    P.o_et = take(nq * 32);
    P.o_fin = take(nq * sizeof(pc_final));
    // each query's count staircase (rows of 2S integers from 0)
    P.roff.clear();
    P.o_roff.resize(nq);
    P.cells.resize(nq);
    for (uint32_t i = 0; i < nq; i++) {
        const BatchQuery &b = R[i];
        P.o_roff[i] = P.roff.size();
        uint64_t off = 0;
        P.roff.push_back(0);
        for (uint64_t r = 0; r < b.nseg; r++) {
            off += row_len(b.x, b.c, b.nb, r * (2ull << kBatchLog2S));
            P.roff.push_back(off);
        }
        P.cells[i] = off;
    }
    P.o_q.resize(nq);
    for (uint32_t i = 0; i < nq; i++)
        P.o_q[i] = take(query_chunk(R[i], P.cells[i]));

    P.blk.clear();
    auto table = [&](auto nblocks_of, uint32_t *nblocks) {
        const size_t at = P.blk.size();
        std::vector<uint32_t> first(nq + 1);
        uint32_t nbk = 0;
        for (uint32_t i = 0; i < nq; i++) {
            first[i] = nbk;
            nbk += std::max<uint32_t>(1, nblocks_of(R[i]));
        }
        first[nq] = nbk;
        for (uint32_t i = 0; i < nq; i++)
            for (uint32_t k = first[i]; k < first[i + 1]; k++)
                P.blk.push_back(i);
        P.blk.insert(P.blk.end(), first.begin(), first.end());
        *nblocks = nbk;
        return at; // q at [at, at + nbk), first at [at + nbk, at + nbk + nq + 1)
    };
    P.t_xb = table(
        [](const BatchQuery &b) { return (uint32_t)std::min<uint64_t>(64, (b.a + 2 + 255) / 256); },
        &P.nb_xb);
    P.t_s1 = table(
        [](const BatchQuery &b) { return (uint32_t)std::min<uint64_t>(64, b.y / 4096 + 1); },
        &P.nb_s1);
    P.t_ez = table(
        [](const BatchQuery &b) { return (uint32_t)std::min<uint64_t>(1024, b.y / 4096 + 1); },
        &P.nb_ez);
    P.t_sc = table([](const BatchQuery &b) { return (b.ncol + 255) / 256; }, &P.nb_sc);

    // sieve tiles, largest queries first, each query's low (leaf-dense) segments first
    std::vector<uint32_t> order(nq);
    for (uint32_t i = 0; i < nq; i++)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t u, uint32_t v) { return R[u].bytes() > R[v].bytes(); });
    P.tiles.clear();
    for (uint32_t i : order)
        for (uint64_t sg = 0; sg < R[i].nseg; sg++)
            P.tiles.push_back(pc_tile{(uint32_t)sg, 0, R[i].ncol, i});
}

// The round's per-query scalars, with their arrays carved out of the arena at
// base; roff: the device copy of P.roff.
void round_queries(const std::vector<BatchQuery> &R, const RoundPlan &P, char *base,
                   const uint64_t *roff, const pc_tables &T, std::vector<pc_query> &Qv)
{
    const uint32_t nq = (uint32_t)R.size();
    const uint64_t S = 1ull << kBatchLog2S;
    pc_sums *sums = reinterpret_cast<pc_sums *>(base + P.o_sums);
    Qv.assign(nq, pc_query{});
    for (uint32_t i = 0; i < nq; i++) {
        const BatchQuery &b = R[i];
        pc_query &Q = Qv[i];
        size_t o = P.o_q[i];
        const size_t o_end = P.o_q[i] + query_chunk(b, P.cells[i]);
        auto carve = [&](size_t bytes) {
            char *p = base + o;
            o += r256(bytes);
            if (o > o_end) // query_chunk and these carves must agree
                fail(PC_EINTERNAL, "batch arena layout");
            return p;
        };
        const uint64_t na = b.a + 2;
        Q.x = b.x;
        Q.x_hi = 0;
        Q.xd = (double)b.x;
        Q.y = b.y;
        Q.z = b.z;
        Q.y1 = b.y + 1;
        Q.recip_y1 = pc_recip(b.y + 1);
        Q.sqrtx = pc_isqrt(b.x);
        Q.sqrty = pc_isqrt(b.y);
        Q.Qc = T.Qc;
        Q.recip_Qc = pc_recip(T.Qc);
        Q.c = b.c;
        Q.a = (uint32_t)b.a;
        Q.bmax = (uint32_t)b.bmax;
        Q.nb = b.nb;
        Q.ncol = b.ncol;
        Q.kx = (uint32_t)b.kx;
        Q.Xb = Q.Xb_w = reinterpret_cast<uint64_t *>(carve(na * 8));
        Q.Ub = Q.Ub_w = reinterpret_cast<ulonglong2 *>(carve(na * 16));
        Q.e_start = reinterpret_cast<uint64_t *>(carve(na * 8));
        Q.e_count = reinterpret_cast<uint64_t *>(carve(na * 8));
        Q.e_off = reinterpret_cast<uint64_t *>(carve(na * 8));
        Q.e_scount = reinterpret_cast<uint64_t *>(carve(na * 8));
        Q.e_clu = reinterpret_cast<uint4 *>(carve(na * 16));
        Q.Xd = reinterpret_cast<double *>(carve(na * 8));
        Q.Xbh = nullptr; // batch queries lie below 2^64
        const size_t nband = b.a / PC_EZ_BAND + 1;
        Q.e_bk = reinterpret_cast<uint32_t *>(carve(2 * nband * 4));
        Q.e_boff = reinterpret_cast<uint64_t *>(carve(2 * nband * 8));
        Q.row_off = roff + P.o_roff[i];
        Q.cnt = reinterpret_cast<uint32_t *>(carve(P.cells[i] * 4));
        Q.wgt = reinterpret_cast<int32_t *>(carve(P.cells[i] * 4));
        Q.cntP = reinterpret_cast<uint32_t *>(carve(b.nseg * 4));
        Q.wP = reinterpret_cast<int32_t *>(carve(b.nseg * 4));
        Q.carryP = nullptr;
        Q.e_total = reinterpret_cast<uint64_t *>(base + P.o_et) + 4 * i;
        Q.sums = sums + i;
        Q.carry = nullptr;
        Q.nseg = b.nseg;
        Q.sieve_end = b.nseg * 2 * S;
    }
}

// The round's kernels on st: clears, set-up, easy leaves, sieve, carries and
// combination into the pc_final array of the arena.  qs, tiles and bk hold
// the uploaded Qv, P.tiles and P.blk.
void round_launches(const RoundPlan &P, uint32_t nq, char *base, const pc_tables &T,
                    const pc_query *qs, const pc_tile *tiles, const uint32_t *bk, int32_t *err,
                    const Knobs &K, hipStream_t st)
{
    pc_sums *sums = reinterpret_cast<pc_sums *>(base + P.o_sums);
    pc_final *fin = reinterpret_cast<pc_final *>(base + P.o_fin);
    hipck(pc_launch_fill_u64(reinterpret_cast<uint64_t *>(err), 1, 0, st), "fill");
    hipck(pc_launch_fill_u64(reinterpret_cast<uint64_t *>(sums), nq * sizeof(pc_sums) / 8, 0, st),
          "fill");
    // results cleared (ok = 0): a read-back that overtook the combination
    // shows up as an error instead of the arena's previous values
    static_assert(sizeof(pc_final) % 8 == 0, "pc_final is filled as u64 words");
    hipck(pc_launch_fill_u64(reinterpret_cast<uint64_t *>(fin), nq * sizeof(pc_final) / 8, 0, st),
          "fill");
    hipck(pc_launch_batch_setup(T, qs, bk + P.t_xb, bk + P.t_xb + P.nb_xb, P.nb_xb, bk + P.t_s1,
                                bk + P.t_s1 + P.nb_s1, P.nb_s1, nq, st),
          "batch set-up");
    hipck(pc_launch_batch_easy(T, qs, bk + P.t_ez, bk + P.t_ez + P.nb_ez, P.nb_ez, st),
          "batch easy");
    pc_sieve_args A{};
    A.T = T;
    A.Qs = qs;
    A.tiles = tiles;
    A.ntiles = (uint32_t)P.tiles.size();
    A.err = err;
    hipck(pc_launch_sieve(A, kBatchLog2S, kBatchWG, PC_MODE_TALLY | (K.batch ? 0 : 0x100), st),
          "batch sieve");
    hipck(pc_launch_batch_finish(qs, bk + P.t_sc, bk + P.t_sc + P.nb_sc, P.nb_sc, nq, fin, st),
          "batch finish");
}

// Queue one round (sl.R) on the slot's stream: its kernels (as a HIP graph
// unless use_graph is false), then the copies of the results into pinned
// memory and the slot's completion event.
void submit_round(BatchSlot &sl, const Knobs &K, bool use_graph)
{
    const std::vector<BatchQuery> &R = sl.R;
    const uint32_t nq = (uint32_t)R.size();
    hipStream_t st = sl.st ? sl.st : g_stream;
    const pc_tables T = tables_view(kWheelC);
    RoundPlan &P = sl.plan;
    plan_round(R, P);
    slot_ensure(sl, sl.arena, P.arena, "batch arena");
    slot_ensure(sl, sl.roff, P.roff.size() * 8, "batch row offsets");
    char *base = static_cast<char *>(sl.arena.p);
    round_queries(R, P, base, ptr<uint64_t>(sl.roff), T, sl.Qv);

    slot_ensure(sl, sl.qs, nq * sizeof(pc_query), "batch queries");
    slot_ensure(sl, sl.tiles, P.tiles.size() * sizeof(pc_tile), "batch tiles");
    slot_ensure(sl, sl.blk, P.blk.size() * 4, "batch blocks");
    slot_ensure(sl, sl.err, 8, "error flag");
    if (sl.h_fin_cap < nq) {
        if (sl.h_fin)
            (void)hipHostFree(sl.h_fin);
        sl.h_fin = nullptr;
        hipck(hipHostMalloc((void **)&sl.h_fin, nq * sizeof(pc_final)), "hipHostMalloc");
        sl.h_fin_cap = nq;
    }
    if (!sl.h_err)
        hipck(hipHostMalloc((void **)&sl.h_err, 8), "hipHostMalloc");
    memset(sl.h_fin, 0, nq * sizeof(pc_final)); // ok = 0 until this round's copy lands
    if (!sl.done)
        hipck(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming), "hipEventCreate");
    hipck(hipMemcpyAsync(sl.qs.p, sl.Qv.data(), nq * sizeof(pc_query), hipMemcpyHostToDevice, st),
          "H2D");
    hipck(hipMemcpyAsync(sl.tiles.p, P.tiles.data(), P.tiles.size() * sizeof(pc_tile),
                         hipMemcpyHostToDevice, st),
          "H2D");
    hipck(hipMemcpyAsync(sl.blk.p, P.blk.data(), P.blk.size() * 4, hipMemcpyHostToDevice, st),
          "H2D");
    hipck(hipMemcpyAsync(sl.roff.p, P.roff.data(), P.roff.size() * 8, hipMemcpyHostToDevice, st),
          "H2D");
    auto launches = [&]() {
        round_launches(P, nq, base, T, ptr<pc_query>(sl.qs), ptr<pc_tile>(sl.tiles),
                       ptr<uint32_t>(sl.blk), ptr<int32_t>(sl.err), K, st);
    };
    if (use_graph) {
        hipck(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        try {
            launches();
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(st, &g);
            if (g)
                (void)hipGraphDestroy(g);
            throw;
        }
        hipck(hipStreamEndCapture(st, &sl.graph), "hipStreamEndCapture");
        hipck(hipGraphInstantiate(&sl.exec, sl.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        hipck(hipGraphLaunch(sl.exec, st), "hipGraphLaunch");
    } else {
        launches();
    }
    const pc_final *fin = reinterpret_cast<const pc_final *>(base + P.o_fin);
    hipck(hipMemcpyAsync(sl.h_fin, fin, nq * sizeof(pc_final), hipMemcpyDeviceToHost, st), "D2H");
    hipck(hipMemcpyAsync(sl.h_err, sl.err.p, 4, hipMemcpyDeviceToHost, st), "D2H");
    hipck(hipEventRecord(sl.done, st), "hipEventRecord");
    sl.busy = true;
}

// After the slot's event: results to out[], graph released, slot free.
void collect_round(BatchSlot &sl, uint64_t *out)
{
    if (sl.exec)
        (void)hipGraphExecDestroy(sl.exec);
    if (sl.graph)
        (void)hipGraphDestroy(sl.graph);
    sl.exec = nullptr;
    sl.graph = nullptr;
    sl.busy = false;
    if (*sl.h_err)
        fail(PC_EINTERNAL, "a leaf or P2 quotient fell outside its segment (batch)");
    for (size_t i = 0; i < sl.R.size(); i++) {
        if (sl.h_fin[i].ok != 1)
            fail(PC_EINTERNAL, "pi(x) outside [0, 2^64), or the round's results were not read "
                               "back in order (batch)");
        out[sl.R[i].idx] = sl.h_fin[i].pi;
    }
}

BatchSlot g_slot; // the synchronous batch path's slot, on the library stream

// y of every query x >= kSmallX, and the pi-table limit and largest y they need.
struct QueryYs {
    std::vector<uint64_t> ys;
    uint64_t need = kSmallX, ymax = 0;
};

QueryYs query_ys(const uint64_t *xs, size_t n, double alpha)
{
    if (std::isnan(alpha) || alpha < 0)
        fail(PC_EINVAL, "alpha must be >= 0 (0 = tuned)");
    QueryYs Y;
    Y.ys.assign(n, 0);
    for (size_t i = 0; i < n; i++) {
        if (xs[i] < kSmallX)
            continue;
        Y.ys[i] = choose_y(xs[i], alpha > 0 ? alpha : default_batch_alpha(xs[i]));
        Y.need = std::max<uint64_t>({Y.need, pc_isqrt(xs[i]), Y.ys[i]});
        Y.ymax = std::max(Y.ymax, Y.ys[i]);
    }
    return Y;
}

// The points whose pi the planner needs: per query y, isqrt x, isqrt(x / y)
// (x itself for x < kSmallX, whose pi is the answer).
std::vector<uint64_t> query_points(const uint64_t *xs, size_t n, const QueryYs &Y)
{
    std::vector<uint64_t> pts;
    pts.reserve(3 * n);
    for (size_t i = 0; i < n; i++) {
        const bool small = xs[i] < kSmallX;
        pts.push_back(small ? xs[i] : Y.ys[i]);
        pts.push_back(small ? 0 : pc_isqrt(xs[i]));
        pts.push_back(small ? 0 : pc_isqrt(xs[i] / Y.ys[i]));
    }
    return pts;
}

// Parameters of every query x >= kSmallX from the looked-up pi values (small x
// are answered into out); *amax = the largest a.
std::vector<BatchQuery> query_params(const uint64_t *xs, size_t n, const QueryYs &Y,
                                     const std::vector<uint64_t> &lk, uint64_t *out,
                                     uint64_t *amax)
{
    *amax = 0;
    std::vector<BatchQuery> big;
    for (size_t i = 0; i < n; i++) {
        if (xs[i] < kSmallX) {
            out[i] = lk[3 * i];
            continue;
        }
        BatchQuery b{};
        b.x = xs[i];
        b.y = Y.ys[i];
        b.a = lk[3 * i];
        b.kx = lk[3 * i + 1];
        b.bmax = lk[3 * i + 2];
        b.z = xs[i] / Y.ys[i];
        b.c = (uint32_t)std::min<uint64_t>(kWheelC, b.a);
        b.nb = b.bmax > b.c ? (uint32_t)(b.bmax - b.c) : 0;
        b.ncol = b.nb + 1;
        b.nseg = b.z / (2ull << kBatchLog2S) + 1;
        b.idx = i;
        *amax = std::max(*amax, b.a);
        big.push_back(b);
    }
    return big;
}

// Parameters of every query x >= kSmallX (small x are answered into out),
// with the tables all of them need.
std::vector<BatchQuery> plan_queries(const uint64_t *xs, size_t n, double alpha, uint64_t *out)
{
    const QueryYs Y = query_ys(xs, n, alpha);
    init_stream();
    ensure_pi(std::max<uint64_t>(Y.need, 1024) + 1);
    uint64_t amax = 0;
    std::vector<BatchQuery> big = query_params(xs, n, Y, lookup(query_points(xs, n, Y)), out,
                                               &amax);
    if (!big.empty()) {
        ensure_mulpf(Y.ymax);
        ensure_recip(amax + 1);
        ensure_wheel(kWheelC);
        hipck(hipStreamSynchronize(g_stream), "sync");
    }
    return big;
}

void run_batch(const uint64_t *xs, size_t n, const Knobs &K, double alpha, bool use_graph,
               uint64_t *out)
{
    const std::vector<BatchQuery> big = plan_queries(xs, n, alpha, out);
    // rounds in input order, each within the carry budget
    BatchSlot &sl = g_slot;
    auto flush = [&]() {
        if (sl.R.empty())
            return;
        submit_round(sl, K, use_graph);
        hipck(hipEventSynchronize(sl.done), "hipEventSynchronize");
        collect_round(sl, out);
        sl.R.clear();
        sl.bytes = 0;
    };
    for (const BatchQuery &b : big) {
        if (b.bytes() > K.carry_budget) { // alone, windowed
            flush();
            pc_result r;
            run_query(b.x, b.y, K, &r);
            out[b.idx] = r.pi;
            continue;
        }
        if (sl.bytes + b.bytes() > K.carry_budget || sl.R.size() >= 65536)
            flush();
        sl.R.push_back(b);
        sl.bytes += b.bytes();
    }
    flush();
}

// ---------------------------------------------------------------------------
// Batches in caller memory.  The caller's workspace holds, in this order, each
// round's uploaded arrays (query scalars, tiles, block tables, output
// positions), the results known on the host ((position, value) pairs: x below
// the sieve threshold, and queries too large for a round, computed windowed
// during the call), the error flag, and one round arena that the rounds reuse
// one after another in stream order.
// ---------------------------------------------------------------------------
struct AsyncRound {
    std::vector<BatchQuery> R;
    RoundPlan P;
    size_t o_qs = 0, o_tiles = 0, o_blk = 0, o_pos = 0, o_roff = 0;
};

struct AsyncPlan {
    std::vector<uint64_t> known;       // results of x < kSmallX (by position)
    std::vector<size_t> known_idx;     // positions answered on the host
    std::vector<BatchQuery> windowed;  // computed during the call, windowed
    std::vector<AsyncRound> rounds;
    size_t o_kv = 0, nkv = 0, o_err = 0, o_arena = 0, total = 0;
};

// The rounds and the workspace layout of a caller-memory batch, from the
// planned queries (A.known holds the answers of x < kSmallX).
void async_layout(const uint64_t *xs, size_t n, const std::vector<BatchQuery> &big,
                  const Knobs &K, AsyncPlan &A);

void async_plan(const uint64_t *xs, size_t n, const Knobs &K, AsyncPlan &A)
{
    A.known.assign(n, 0);
    const std::vector<BatchQuery> big = plan_queries(xs, n, 0.0, A.known.data());
    async_layout(xs, n, big, K, A);
}

void async_layout(const uint64_t *xs, size_t n, const std::vector<BatchQuery> &big,
                  const Knobs &K, AsyncPlan &A)
{
    for (size_t i = 0; i < n; i++)
        if (xs[i] < kSmallX)
            A.known_idx.push_back(i);
    // the rounds of the synchronous path: in input order within the carry budget
    std::vector<BatchQuery> cur;
    uint64_t bytes = 0;
    auto flush = [&]() {
        if (cur.empty())
            return;
        A.rounds.emplace_back();
        A.rounds.back().R.swap(cur);
        bytes = 0;
    };
    for (const BatchQuery &b : big) {
        if (b.bytes() > K.carry_budget) {
            A.windowed.push_back(b);
            continue;
        }
        if (bytes + b.bytes() > K.carry_budget || cur.size() >= 65536)
            flush();
        cur.push_back(b);
        bytes += b.bytes();
    }
    flush();
    A.nkv = A.known_idx.size() + A.windowed.size();
    size_t tot = 0, arena = 0;
    auto take = [&](size_t bytes) {
        const size_t o = tot;
        tot += r256(bytes);
        return o;
    };
    for (AsyncRound &r : A.rounds) {
        plan_round(r.R, r.P);
        r.o_qs = take(r.R.size() * sizeof(pc_query));
        r.o_tiles = take(r.P.tiles.size() * sizeof(pc_tile));
        r.o_blk = take(r.P.blk.size() * 4);
        r.o_pos = take(r.R.size() * 8);
        r.o_roff = take(r.P.roff.size() * 8);
        arena = std::max(arena, r.P.arena);
    }
    A.o_kv = take(A.nkv * 16);
    A.o_err = take(8);
    A.o_arena = take(arena);
    A.total = A.rounds.empty() ? A.o_err : tot; // no round: no flag, no arena
}

uint64_t *g_async_host = nullptr; // pinned staging for xs and the upload
size_t g_async_host_cap = 0;

void *async_staging(size_t bytes)
{
    if (g_async_host_cap < bytes) {
        if (g_async_host)
            (void)hipHostFree(g_async_host);
        g_async_host = nullptr;
        g_async_host_cap = 0;
        const size_t cap = std::max<size_t>(bytes, 1 << 16);
        hipck(hipHostMalloc((void **)&g_async_host, cap), "hipHostMalloc");
        g_async_host_cap = cap;
    }
    return g_async_host;
}

void async_queue(const AsyncPlan &A, const std::vector<ulonglong2> &kv, char *img, char *ws,
                 uint64_t *d_out, const Knobs &K, hipStream_t st);

void run_batch_async(const uint64_t *d_xs, size_t n, uint64_t *d_out, void *d_ws, size_t ws_bytes,
                     hipStream_t st)
{
    init_stream();
    const Knobs K;
    // the queries, once the stream's earlier work has produced them
    uint64_t *hx = static_cast<uint64_t *>(async_staging(n * 8));
    hipck(hipMemcpyAsync(hx, d_xs, n * 8, hipMemcpyDeviceToHost, st), "D2H");
    hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
    const std::vector<uint64_t> xs(hx, hx + n);
    AsyncPlan A;
    async_plan(xs.data(), n, K, A);
    if (A.total > ws_bytes || (A.total > 0 && !d_ws))
        fail(PC_ENOMEM, "workspace of " + std::to_string(ws_bytes) + " bytes; these queries need " +
                            std::to_string(A.total) + " (pc_workspace_bytes)");
    std::vector<ulonglong2> kv;
    kv.reserve(A.nkv);
    for (size_t i : A.known_idx)
        kv.push_back(ulonglong2{i, A.known[i]});
    for (const BatchQuery &b : A.windowed) {
        pc_result r;
        run_query(b.x, b.y, K, &r);
        kv.push_back(ulonglong2{b.idx, r.pi});
    }
    async_queue(A, kv, static_cast<char *>(async_staging(A.o_err)), static_cast<char *>(d_ws),
                d_out, K, st);
    hipEvent_t e = nullptr;
    if (!g_async_spare.empty()) {
        e = g_async_spare.back();
        g_async_spare.pop_back();
    } else {
        hipck(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    }
    g_async_live.push_back(e);
    hipck(hipEventRecord(e, st), "hipEventRecord");
    // forget the batches that have finished
    for (size_t i = 0; i < g_async_live.size();)
        if (g_async_live[i] != e && hipEventQuery(g_async_live[i]) == hipSuccess) {
            g_async_spare.push_back(g_async_live[i]);
            g_async_live[i] = g_async_live.back();
            g_async_live.pop_back();
        } else {
            i++;
        }
}

// Queue the rounds of plan A on st with the workspace ws: one upload of
// everything before the error flag, staged in img (host, A.o_err bytes; free
// again when this returns, since the upload is waited for), the results known
// on the host (kv), then each round's kernels and its results into d_out.
void async_queue(const AsyncPlan &A, const std::vector<ulonglong2> &kv, char *img, char *ws,
                 uint64_t *d_out, const Knobs &K, hipStream_t st)
{
    char *arena = ws + A.o_arena;
    const pc_tables T = tables_view(kWheelC);
    std::vector<pc_query> Qv;
    for (const AsyncRound &r : A.rounds) {
        round_queries(r.R, r.P, arena, reinterpret_cast<const uint64_t *>(ws + r.o_roff), T, Qv);
        memcpy(img + r.o_roff, r.P.roff.data(), r.P.roff.size() * 8);
        memcpy(img + r.o_qs, Qv.data(), Qv.size() * sizeof(pc_query));
        memcpy(img + r.o_tiles, r.P.tiles.data(), r.P.tiles.size() * sizeof(pc_tile));
        memcpy(img + r.o_blk, r.P.blk.data(), r.P.blk.size() * 4);
        uint64_t *pos = reinterpret_cast<uint64_t *>(img + r.o_pos);
        for (size_t i = 0; i < r.R.size(); i++)
            pos[i] = r.R[i].idx;
    }
    if (!kv.empty())
        memcpy(img + A.o_kv, kv.data(), kv.size() * 16);
    hipck(hipMemcpyAsync(ws, img, A.o_err, hipMemcpyHostToDevice, st), "H2D");
    hipck(hipStreamSynchronize(st), "hipStreamSynchronize"); // the staging is free again
    hipck(pc_launch_scatter_u64(reinterpret_cast<const ulonglong2 *>(ws + A.o_kv), kv.size(),
                                d_out, st),
          "results");
    int32_t *err = reinterpret_cast<int32_t *>(ws + A.o_err);
    for (const AsyncRound &r : A.rounds) {
        const uint32_t nq = (uint32_t)r.R.size();
        round_launches(r.P, nq, arena, T, reinterpret_cast<const pc_query *>(ws + r.o_qs),
                       reinterpret_cast<const pc_tile *>(ws + r.o_tiles),
                       reinterpret_cast<const uint32_t *>(ws + r.o_blk), err, K, st);
        hipck(pc_launch_batch_out(reinterpret_cast<const pc_final *>(arena + r.P.o_fin),
                                  reinterpret_cast<const uint64_t *>(ws + r.o_pos), nq, err, d_out,
                                  st),
              "results");
    }
}

// ---------------------------------------------------------------------------
// The caller-memory batch without any allocation.  The workspace is one fixed
// device array of the library (every device it runs on holds its own copy
// until the process ends), and the shared device tables must already cover
// the queries: the call never builds or grows them.  The array's name is a
// host-side stand-in; its device address comes from hipGetSymbolAddress once
// per device, and only that address is used.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = PC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::vector<void *> g_scratch; // device address of scratch, by device ordinal

char *scratch_ptr()
{
    int dev = 0;
    hipck(hipGetDevice(&dev), "hipGetDevice");
    if ((size_t)dev >= g_scratch.size())
        g_scratch.resize((size_t)dev + 1, nullptr);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        hipck(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = p;
    }
    return static_cast<char *>(g_scratch[dev]);
}

void run_batch_noalloc(const uint64_t *d_xs, size_t n, uint64_t *d_out, hipStream_t st)
{
    Tables &T = g_T;
    if (!g_stream || !T.base_ok || !T.wheel_ok[kWheelC])
        fail(PC_ERANGE, "the device tables are not built: call pc_workspace_bytes (or any "
                        "batch) with these queries first");
    if (n > kScratchBytes / 48)
        fail(PC_ENOMEM, "more queries than the scratch array holds (" +
                            std::to_string(kScratchBytes / 48) + ")");
    char *ws = scratch_ptr();
    std::vector<uint64_t> xs(n);
    hipck(hipMemcpyAsync(xs.data(), d_xs, n * 8, hipMemcpyDeviceToHost, st), "D2H");
    hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
    const QueryYs Y = query_ys(xs.data(), n, 0.0);
    if (T.pi_limit < std::max<uint64_t>(Y.need, 1024) + 1 || T.y_limit < Y.ymax)
        fail(PC_ERANGE, "the device tables do not cover these queries: call "
                        "pc_workspace_bytes (or any batch) with them first");
    // pi at the planning points, staged in the scratch array
    const std::vector<uint64_t> pts = query_points(xs.data(), n, Y);
    uint64_t *d_in = reinterpret_cast<uint64_t *>(ws), *d_lk = d_in + pts.size();
    std::vector<uint64_t> lk(pts.size());
    hipck(hipMemcpyAsync(d_in, pts.data(), pts.size() * 8, hipMemcpyHostToDevice, st), "H2D");
    hipck(pc_launch_lookup(ptr<uint2>(T.pitab), d_in, (uint32_t)pts.size(), d_lk, st), "lookup");
    hipck(hipMemcpyAsync(lk.data(), d_lk, lk.size() * 8, hipMemcpyDeviceToHost, st), "D2H");
    hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
    AsyncPlan A;
    A.known.assign(n, 0);
    uint64_t amax = 0;
    const std::vector<BatchQuery> big = query_params(xs.data(), n, Y, lk, A.known.data(), &amax);
    if (!big.empty() && T.recip_n < amax + 1)
        fail(PC_ERANGE, "the device tables do not cover these queries: call "
                        "pc_workspace_bytes (or any batch) with them first");
    Knobs K;
    K.carry_budget = kScratchBytes / 2; // one round's counts and weights
    async_layout(xs.data(), n, big, K, A);
    if (!A.windowed.empty())
        fail(PC_ERANGE, "x = " + std::to_string(A.windowed[0].x) + " needs " +
                            std::to_string(A.windowed[0].bytes()) +
                            " bytes of sieve counts, more than a round of the scratch array");
    if (A.total > kScratchBytes)
        fail(PC_ENOMEM, "these queries need " + std::to_string(A.total) +
                            " bytes of workspace; the scratch array has " +
                            std::to_string(kScratchBytes));
    std::vector<ulonglong2> kv;
    kv.reserve(A.nkv);
    for (size_t i : A.known_idx)
        kv.push_back(ulonglong2{i, A.known[i]});
    std::vector<char> img(A.o_err);
    async_queue(A, kv, img.data(), ws, d_out, K, st);
    // wait: the next call reuses the array, and the tables must outlive the kernels
    int32_t err = 0;
    if (!A.rounds.empty())
        hipck(hipMemcpyAsync(&err, ws + A.o_err, 4, hipMemcpyDeviceToHost, st), "D2H");
    hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (err)
        fail(PC_EINTERNAL, "a leaf or P2 quotient fell outside its segment (batch)");
}

// ---------------------------------------------------------------------------
// Serving: an open-loop request stream replayed in real time.  Requests that
// have arrived wait in a FIFO; whenever a slot (a stream with its own round
// buffers) is free and the device-memory budget allows, the waiting requests
// form a round that goes to the device at once, so rounds of later arrivals
// overlap the ones already running.  A request whose counts exceed a round's
// budget runs alone through the windowed path on a worker thread (the library
// stream), beside the rounds.  x < 2^20 is answered from the pi table on
// arrival.  Latency = completion - arrival, on the host clock.
// ---------------------------------------------------------------------------
void run_serve(const uint64_t *xs, const double *arr, size_t n, const pc_serve_config &C,
               uint64_t *pi_out, double *lat_out, pc_serve_stats *stats)
{
    for (size_t i = 0; i < n; i++) {
        if (!(arr[i] >= 0) || !std::isfinite(arr[i]))
            fail(PC_EINVAL, "arrival times must be finite and >= 0");
        if (i && arr[i] < arr[i - 1])
            fail(PC_EINVAL, "arrival times must not decrease");
    }
    const Knobs K;
    const bool use_graph = (C.flags & PC_FLAG_NO_GRAPH) == 0;
    const uint32_t nslot = C.max_inflight ? C.max_inflight : 3;
    const uint32_t maxr = C.max_round ? C.max_round : 4096;
    const uint64_t budget = C.mem_budget ? C.mem_budget : (18ull << 30);
    const uint64_t round_cap = std::min<uint64_t>(K.carry_budget, budget);
    if (nslot > 16)
        fail(PC_EINVAL, "max_inflight must be at most 16");

    std::vector<uint64_t> out(n, 0);
    const std::vector<BatchQuery> big = plan_queries(xs, n, C.alpha, out.data());
    std::vector<int> kind(n, 0); // 0: answered from the table, 1: rounds, 2: windowed
    std::vector<const BatchQuery *> byidx(n, nullptr);
    for (const BatchQuery &b : big) {
        byidx[b.idx] = &b;
        kind[b.idx] = b.bytes() > round_cap ? 2 : 1;
    }
    std::vector<double> tdone(n, -1.0);

    std::vector<BatchSlot> slots(nslot);
    std::mutex m;
    std::condition_variable cv;
    std::deque<size_t> wq;      // windowed requests waiting
    std::vector<size_t> wdone;  // finished, not yet counted
    std::string werr;
    pc_status wst = PC_OK;
    bool stop = false;
    using sclk = std::chrono::steady_clock;
    const auto t0 = sclk::now();
    auto now = [&]() { return std::chrono::duration<double>(sclk::now() - t0).count(); };
    std::thread worker([&]() {
        for (;;) {
            size_t i;
            {
                std::unique_lock<std::mutex> lk(m);
                cv.wait(lk, [&] { return stop || !wq.empty(); });
                if (wq.empty())
                    return;
                i = wq.front();
                wq.pop_front();
            }
            pc_status st = PC_OK;
            std::string msg;
            try {
                pc_result r;
                run_query(xs[i], byidx[i]->y, K, &r);
                out[i] = r.pi;
            } catch (const pc_error &e) {
                st = e.st;
                msg = e.msg;
            } catch (...) {
                st = PC_EINTERNAL;
                msg = "unexpected exception (windowed request)";
            }
            std::lock_guard<std::mutex> lk(m);
            tdone[i] = now();
            wdone.push_back(i);
            if (st != PC_OK && wst == PC_OK) {
                wst = st;
                werr = msg;
            }
        }
    });
    struct Guard { // stop the worker and free the slots however the loop ends
        std::function<void()> f;
        ~Guard() { f(); }
    } guard{[&]() {
        {
            std::lock_guard<std::mutex> lk(m);
            stop = true;
        }
        cv.notify_all();
        if (worker.joinable())
            worker.join();
        for (BatchSlot &sl : slots)
            slot_release(sl);
    }};
    for (BatchSlot &sl : slots)
        hipck(hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking), "hipStreamCreate");

    size_t next = 0, ndone = 0;
    std::deque<size_t> pending;
    uint64_t inflight = 0, rounds = 0, windowed = 0, max_round = 0, max_inflight_seen = 0;
    while (ndone < n) {
        bool moved = false;
        double t = now();
        while (next < n && arr[next] <= t) {
            const size_t i = next++;
            moved = true;
            if (kind[i] == 0) {
                tdone[i] = t;
                ndone++;
            } else if (kind[i] == 2) {
                windowed++;
                std::lock_guard<std::mutex> lk(m);
                wq.push_back(i);
                cv.notify_one();
            } else {
                pending.push_back(i);
            }
        }
        uint32_t busy = 0;
        for (BatchSlot &sl : slots) {
            if (!sl.busy)
                continue;
            const hipError_t e = hipEventQuery(sl.done);
            if (e == hipErrorNotReady) {
                busy++;
                continue;
            }
            hipck(e, "hipEventQuery");
            collect_round(sl, out.data());
            const double tc = now();
            for (const BatchQuery &b : sl.R)
                tdone[b.idx] = tc;
            ndone += sl.R.size();
            inflight -= sl.bytes;
            sl.R.clear();
            sl.bytes = 0;
            moved = true;
        }
        {
            std::lock_guard<std::mutex> lk(m);
            if (wst != PC_OK)
                fail(wst, werr);
            ndone += wdone.size();
            moved |= !wdone.empty();
            wdone.clear();
        }
        for (BatchSlot &sl : slots) {
            if (sl.busy || pending.empty())
                continue;
            const uint64_t room = std::min<uint64_t>(round_cap, budget - inflight);
            while (!pending.empty() && sl.R.size() < maxr) {
                const BatchQuery &b = *byidx[pending.front()];
                if (sl.bytes + b.bytes() > room)
                    break;
                sl.R.push_back(b);
                sl.bytes += b.bytes();
                pending.pop_front();
            }
            if (sl.R.empty())
                break; // the oldest request waits for memory
            submit_round(sl, K, use_graph);
            inflight += sl.bytes;
            rounds++;
            max_round = std::max<uint64_t>(max_round, sl.R.size());
            busy++;
            moved = true;
        }
        max_inflight_seen = std::max<uint64_t>(max_inflight_seen, busy);
        if (!moved) { // nothing to do until a completion or the next arrival
            double wait = 2e-4;
            if (next < n && busy == 0 && pending.empty())
                wait = std::min(wait, std::max(0.0, arr[next] - now()));
            std::this_thread::sleep_for(std::chrono::duration<double>(std::max(wait, 2e-5)));
        }
    }
    const double wall = now();
    for (size_t i = 0; i < n; i++) {
        pi_out[i] = out[i];
        if (lat_out)
            lat_out[i] = tdone[i] - arr[i];
    }
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->wall_s = wall;
        stats->rounds = rounds;
        stats->windowed = windowed;
        stats->max_round_size = max_round;
        stats->max_inflight_seen = max_inflight_seen;
        stats->device_bytes = g_dev_peak.load();
    }
}

} // namespace

extern "C" {

pc_status pc_pi_count(uint64_t x, double alpha, uint64_t *pi_out)
{
    if (!pi_out)
        return PC_EINVAL;
    uint64_t v = 0;
    pc_status st = guarded([&] { pi_one(x, Knobs{}, alpha, nullptr, &v); });
    if (st == PC_OK)
        *pi_out = v;
    return st;
}

pc_status pc_pi_count_ex(uint64_t x, const pc_config *cfg, pc_result *res)
{
    pc_result r;
    uint64_t v = 0;
    pc_status st = guarded([&] {
        Knobs K = knobs_from(cfg);
        if (cfg && (cfg->flags & PC_FLAG_REBUILD_TABLES))
            drop_tables(false);
        pi_one(x, K, cfg ? cfg->alpha : 0.0, &r, &v);
    });
    if (st == PC_OK && res)
        *res = r;
    return st;
}

pc_status pc_pi_count_wide(uint64_t x_lo, uint64_t x_hi, const pc_config *cfg, pc_result *res)
{
    pc_result r;
    uint64_t v = 0;
    pc_status st = guarded([&] {
        if (x_hi > 256 || (x_hi == 256 && x_lo != 0))
            fail(PC_ERANGE, "x must be at most 2^72");
        Knobs K = knobs_from(cfg);
        if (cfg && (cfg->flags & PC_FLAG_REBUILD_TABLES))
            drop_tables(false);
        pi_one(((pc_u128)x_hi << 64) | x_lo, K, cfg ? cfg->alpha : 0.0, &r, &v);
    });
    if (st == PC_OK && res)
        *res = r;
    return st;
}

pc_status pc_decompose(uint64_t x, uint64_t y, const pc_config *cfg, pc_result *res)
{
    pc_result r;
    pc_status st = guarded([&] {
        check_y(x, y);
        Knobs K = knobs_from(cfg);
        if (cfg && (cfg->flags & PC_FLAG_REBUILD_TABLES))
            drop_tables(false);
        run_query(x, y, K, &r);
    });
    if (st == PC_OK && res)
        *res = r;
    return st;
}

pc_status pc_s2_hard(uint64_t x, uint64_t y, uint64_t a, pc_i128 *out)
{
    if (!out)
        return PC_EINVAL;
    pc_result r;
    pc_status st = guarded([&] {
        check_y(x, y);
        init_stream();
        ensure_pi(std::max<uint64_t>(y, 1024) + 1);
        if (lookup({y})[0] != a)
            fail(PC_EINVAL, "a must equal pi(y)");
        run_query(x, y, Knobs{}, &r);
    });
    if (st == PC_OK)
        *out = r.s2_hard;
    return st;
}

pc_status pc_p2(uint64_t x, uint64_t y, uint64_t *out)
{
    if (!out)
        return PC_EINVAL;
    pc_result r;
    pc_status st = guarded([&] {
        check_y(x, y);
        run_query(x, y, Knobs{}, &r);
        if (r.p2.hi != 0)
            fail(PC_EINTERNAL, "P2 outside [0, 2^64)");
    });
    if (st == PC_OK)
        *out = r.p2.lo;
    return st;
}

pc_status pc_pi_count_batch_ex(const uint64_t *xs, size_t n, const pc_config *cfg,
                               uint64_t *pi_out)
{
    if (n == 0)
        return PC_OK;
    if (!xs || !pi_out)
        return PC_EINVAL;
    std::vector<uint64_t> out(n);
    pc_status st = guarded([&] {
        Knobs K = knobs_from(cfg);
        const double alpha = cfg ? cfg->alpha : 0.0;
        const uint32_t flags = cfg ? cfg->flags : 0u;
        if (flags & PC_FLAG_REBUILD_TABLES)
            drop_tables(false);
        if (flags & PC_FLAG_BATCH_SEQUENTIAL) {
            if (std::isnan(alpha) || alpha < 0)
                fail(PC_EINVAL, "alpha must be >= 0 (0 = tuned)");
            for (size_t i = 0; i < n; i++)
                pi_one(xs[i], K, alpha, nullptr, &out[i]);
        } else {
            run_batch(xs, n, K, alpha, (flags & PC_FLAG_NO_GRAPH) == 0, out.data());
        }
    });
    if (st == PC_OK)
        memcpy(pi_out, out.data(), n * 8);
    return st;
}

pc_status pc_serve(const uint64_t *xs, const double *arrival_s, size_t n,
                   const pc_serve_config *cfg, uint64_t *pi_out, double *latency_s_out,
                   pc_serve_stats *stats)
{
    if (n == 0)
        return PC_OK;
    if (!xs || !arrival_s || !pi_out)
        return PC_EINVAL;
    pc_serve_config C{};
    if (cfg)
        C = *cfg;
    std::vector<uint64_t> out(n);
    std::vector<double> lat(n);
    pc_serve_stats st{};
    pc_status s = guarded([&] { run_serve(xs, arrival_s, n, C, out.data(), lat.data(), &st); });
    if (s == PC_OK) {
        memcpy(pi_out, out.data(), n * 8);
        if (latency_s_out)
            memcpy(latency_s_out, lat.data(), n * 8);
        if (stats)
            *stats = st;
    }
    return s;
}

pc_status pc_pi_count_batch(const uint64_t *xs, size_t n, uint64_t *pi_out)
{
    return pc_pi_count_batch_ex(xs, n, nullptr, pi_out);
}

size_t pc_workspace_bytes(const uint64_t *xs, size_t n)
{
    if (n == 0)
        return 0;
    if (!xs) {
        t_err = "xs is null";
        return SIZE_MAX;
    }
    size_t bytes = SIZE_MAX;
    const pc_status st = guarded([&] {
        AsyncPlan A;
        async_plan(xs, n, Knobs{}, A);
        bytes = A.total;
    });
    return st == PC_OK ? bytes : SIZE_MAX;
}

pc_status pc_pi_count_batch_noalloc(const uint64_t *d_xs, size_t n, uint64_t *d_out,
                                    void *hip_stream)
{
    if (n == 0)
        return PC_OK;
    if (!d_xs || !d_out) {
        t_err = "d_xs and d_out must be device pointers";
        return PC_EINVAL;
    }
    return guarded(
        [&] { run_batch_noalloc(d_xs, n, d_out, static_cast<hipStream_t>(hip_stream)); });
}

pc_status pc_pi_count_batch_async(const uint64_t *d_xs, size_t n, uint64_t *d_out, void *d_ws,
                                  size_t ws_bytes, void *hip_stream)
{
    if (n == 0)
        return PC_OK;
    if (!d_xs || !d_out) {
        t_err = "d_xs and d_out must be device pointers";
        return PC_EINVAL;
    }
    return guarded([&] {
        run_batch_async(d_xs, n, d_out, d_ws, ws_bytes, static_cast<hipStream_t>(hip_stream));
    });
}

pc_status pc_read_table(int which, uint64_t lo, uint64_t n, void *out)
{
    if (n == 0)
        return PC_OK;
    if (!out) {
        t_err = "out must not be null";
        return PC_EINVAL;
    }
    return guarded([&] {
        init_stream();
        Tables &T = g_T;
        const uint64_t last = lo + n - 1;
        if (last < lo)
            fail(PC_EINVAL, "range wraps around");
        if (which == PC_TABLE_PRIMES) {
            if (lo < 1)
                fail(PC_EINVAL, "primes are numbered from 1");
            uint64_t lim = 1024;
            for (;;) { // grow the pi table until it holds p_last
                ensure_pi(lim);
                if (T.nprimes >= last)
                    break;
                if (T.pi_limit >= 0xFFFFFFFFull)
                    fail(PC_EINVAL, "p_k beyond 2^32 requested");
                lim = std::min<uint64_t>(2 * T.pi_limit + 2, 0xFFFFFFFFull);
            }
            if (last >= T.k32) // the 32-bit array ends below 2^32
                fail(PC_EINVAL, "p_k beyond 2^32 requested");
            hipck(hipMemcpyAsync(out, ptr<uint32_t>(T.primes) + lo, n * 4, hipMemcpyDeviceToHost,
                                 g_stream),
                  "D2H");
            hipck(hipStreamSynchronize(g_stream), "sync");
        } else if (which == PC_TABLE_PI) {
            if (last > 0xFFFFFFFFull)
                fail(PC_EINVAL, "pi table ends below 2^32");
            ensure_pi(std::max<uint64_t>(last, 1024));
            std::vector<uint64_t> pts(n);
            for (uint64_t i = 0; i < n; i++)
                pts[i] = lo + i;
            const std::vector<uint64_t> v = lookup(pts);
            memcpy(out, v.data(), n * 8);
        } else if (which == PC_TABLE_MULPF) {
            if (last > (1ull << 31) - 2)
                fail(PC_EINVAL, "mu*lpf table ends at 2^31 - 2");
            ensure_mulpf(std::max<uint64_t>(last, 1));
            hipck(hipMemcpyAsync(out, ptr<int32_t>(T.mulpf) + lo, n * 4, hipMemcpyDeviceToHost,
                                 g_stream),
                  "D2H");
            hipck(hipStreamSynchronize(g_stream), "sync");
        } else {
            fail(PC_EINVAL, "unknown table");
        }
    });
}

pc_status pc_phi_seed(uint64_t m, uint32_t c, uint32_t b_hi, uint64_t *out)
{
    if (!out) {
        t_err = "out must not be null";
        return PC_EINVAL;
    }
    if (c < 1 || c > (uint32_t)kWheelC || c > b_hi) {
        t_err = "need 1 <= c <= pc_wheel_c() and c <= b_hi";
        return PC_EINVAL;
    }
    if (m > (1ull << 48) || b_hi >= (1u << 27)) {
        t_err = "need m <= 2^48 and b_hi < 2^27";
        return PC_ERANGE;
    }
    return guarded([&] {
        init_stream();
        Tables &T = g_T;
        // the pi table answers every Legendre lookup (below m^(2/3)) and holds p_{b_hi + 1}
        const uint64_t r = pc_icbrt(m) + 1;
        uint64_t lim = std::max<uint64_t>(r * r, 1024);
        for (;;) {
            ensure_pi(lim);
            if (T.nprimes >= (uint64_t)b_hi + 1)
                break;
            lim = 2 * T.pi_limit + 2;
        }
        ensure_recip((uint64_t)b_hi + 1);
        ensure_wheel(c);
        const uint32_t nb = b_hi - c;
        QueryBufs &B = g_Q;
        ensure(B.seed_term, ((size_t)nb + 1) * 8, "seed terms");
        ensure(B.carry_a, ((size_t)nb + 1) * 8, "carry");
        ensure(B.err, 8, "error flag");
        hipck(pc_launch_fill_u64(ptr<uint64_t>(B.err), 1, 0, g_stream), "fill");
        hipck(pc_launch_seed(tables_view(c), c, m, nb, seed_rec_cols(m, c, nb), T.pi_limit,
                             ptr<int64_t>(B.seed_term), ptr<uint64_t>(B.carry_a),
                             ptr<int32_t>(B.err), g_stream),
              "seeds");
        int32_t err = 0;
        hipck(hipMemcpyAsync(out, B.carry_a.p, ((size_t)nb + 1) * 8, hipMemcpyDeviceToHost,
                             g_stream),
              "D2H");
        hipck(hipMemcpyAsync(&err, B.err.p, 4, hipMemcpyDeviceToHost, g_stream), "D2H");
        hipck(hipStreamSynchronize(g_stream), "sync");
        if (err)
            fail(PC_EINTERNAL, "seeds: pi table too short, stack too deep or a negative phi");
    });
}

int pc_wheel_c(void) { return kWheelC; }

const char *pc_status_str(pc_status s)
{
    switch (s) {
    case PC_OK:
        return "ok";
    case PC_EINVAL:
        return "invalid argument";
    case PC_ERANGE:
        return "out of range";
    case PC_ENOMEM:
        return "out of memory";
    case PC_EDEVICE:
        return "device error";
    case PC_EINTERNAL:
        return "internal error";
    }
    return "unknown status";
}

const char *pc_last_error(void) { return t_err.c_str(); }

void pc_shutdown(void)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    slot_release(g_slot);
    drop_tables(true); // waits for the caller-memory batches still queued
    async_wait_all();
    for (hipEvent_t e : g_async_spare)
        (void)hipEventDestroy(e);
    g_async_spare.clear();
    if (g_async_host)
        (void)hipHostFree(g_async_host);
    g_async_host = nullptr;
    g_async_host_cap = 0;
    drop_query_bufs();
    g_pin.release();
    for (hipStream_t *st : {&g_stream2, &g_stream3})
        if (*st) {
            (void)hipStreamSynchronize(*st);
            (void)hipStreamDestroy(*st);
            *st = nullptr;
        }
    if (g_stream) {
        (void)hipStreamDestroy(g_stream);
        g_stream = nullptr;
    }
    for (hipEvent_t *e : {&g_fork, &g_join, &g_join3})
        if (*e) {
            (void)hipEventDestroy(*e);
            *e = nullptr;
        }
    g_dev_peak = g_dev_bytes.load();
}

} // extern "C"

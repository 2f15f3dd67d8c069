// pc_seed.hip -- the seeds of a sieve started in the middle (Section 4):
// phi(m, b) for one m and every c <= b <= c + nb, computed on their own, so
// that a window of segments starting at m needs nothing from the windows
// before it.
//
// From phi(m, c) (the wheel), eq. (4.1) gives each next column:
//     phi(m, b) = phi(m, b-1) - t_b,   t_b = phi(floor(m / p_b), b-1),
// and the seeds are one prefix sum of the terms.  Each term is taken by the
// rule that fits it (the multifaceted scheme of Section 4):
//   * u = floor(m / p_b) < p_b:      only 1 survives (0 if u = 0), t_b = [u >= 1]
//     (the tail past pi(sqrt m), where each column is the last one less 1);
//   * p_b^2 > u:                     Legendre, t_b = pi(u) - (b-1) + 1, from the
//     pi table (u < m^(2/3) here, inside the table's range);
//   * otherwise:                     eq. (4.1) again on (u, b-1): phi(u, c) less
//     the children (floor(u / p_i), i-1), c < i < b, each resolved the same way
//     depth first.  These are the b with p_b^3 <= m, a few hundred to a few
//     thousand columns; their children's children are dealt out to the
//     threads of one workgroup per column.
// Three launches: the closed terms (one thread per column), the recursive
// terms (one workgroup per column p_b <= icbrt m), and the prefix sum (one
// workgroup).
#include "pc_block.h"
#include "pc_internal.h"

namespace {

constexpr uint32_t SEED_T = 256;    // threads per workgroup of the term kernels
constexpr uint32_t SCAN_T = 1024;   // threads of the prefix-sum workgroup
constexpr int SEED_MAXD = 32;       // depth bound: m <= 2^48 and p_{c+1} >= 3

struct seed_ctx {
    const uint32_t *primes;
    const uint64_t *recip;
    const uint2 *pitab;
    const uint32_t *phitab;
    uint64_t pi_limit;
    uint64_t Qc, rQc;
    uint32_t phiQ, c;
    int32_t *err;
};

// phi(v, c) from the wheel: phi(Q_c, c) per full period plus the table
__device__ __forceinline__ int64_t seed_wheel(const seed_ctx &S, uint64_t v)
{
    const uint64_t q = pc_div(v, S.Qc, S.rQc);
    return (int64_t)(q * S.phiQ + S.phitab[v - q * S.Qc]);
}

// The node (v, k), k >= c, when its value is closed: true and *val set;
// false when eq. (4.1) has to expand it (v >= p_{k+1}^2).
__device__ __forceinline__ bool seed_leaf(const seed_ctx &S, uint64_t v, uint32_t k,
                                          int64_t *val)
{
    if (k <= S.c) {
        *val = seed_wheel(S, v);
        return true;
    }
    const uint64_t q = S.primes[k + 1];
    if (v < q) {
        *val = v ? 1 : 0;
        return true;
    }
    if (v < q * q) {
        if (v > S.pi_limit) { // the caller sized the pi table for every such v
            atomicOr(S.err, 16);
            *val = 0;
        } else {
            *val = (int64_t)pc_pi_lookup(S.pitab, v) - (int64_t)k + 1;
        }
        return true;
    }
    return false;
}

// phi(v, k) by eq. (4.1) depth first, with an explicit stack: a node that
// expands adds phi(v, c) with its sign and pushes its children in turn.
__device__ int64_t seed_phi(const seed_ctx &S, uint64_t v, uint32_t k)
{
    int64_t total;
    if (seed_leaf(S, v, k, &total))
        return total;
    uint64_t sv[SEED_MAXD];
    uint32_t sk[SEED_MAXD], si[SEED_MAXD];
    int d = 0;
    sv[0] = v;
    sk[0] = k;
    si[0] = S.c + 1;
    total = seed_wheel(S, v);
    while (d >= 0) {
        if (si[d] > sk[d]) {
            d--;
            continue;
        }
        const uint32_t i = si[d]++;
        const uint64_t w = pc_div(sv[d], S.primes[i], S.recip[i]);
        const int64_t sgn = (d & 1) ? 1 : -1; // children sit one level down
        int64_t lv;
        if (seed_leaf(S, w, i - 1, &lv)) {
            total += sgn * lv;
        } else {
            if (d + 1 >= SEED_MAXD) {
                atomicOr(S.err, 16);
                return 0;
            }
            d++;
            sv[d] = w;
            sk[d] = i - 1;
            si[d] = S.c + 1;
            total += sgn * seed_wheel(S, w);
        }
    }
    return total;
}

// term[0] = phi(m, c); term[j] = t_{c+j} for 1 <= j <= nb, or phi(u, c) alone
// where the children still have to be taken off (k_seed_rec)
__global__ __launch_bounds__(SEED_T) void k_seed_terms(seed_ctx S, uint64_t m, uint32_t nb,
                                                       int64_t *term)
{
    const uint32_t j = blockIdx.x * SEED_T + threadIdx.x;
    if (j > nb)
        return;
    if (j == 0) {
        term[0] = seed_wheel(S, m);
        return;
    }
    const uint32_t b = S.c + j;
    const uint64_t u = pc_div(m, S.primes[b], S.recip[b]);
    int64_t v;
    term[j] = seed_leaf(S, u, b - 1, &v) ? v : seed_wheel(S, u);
}

// One workgroup per column j = blockIdx.x + 1: if its term expands, the sum
// of its children phi(floor(u / p_i), i-1), c < i < b, comes off the term.
// The threads share the children one level further down, so that no thread
// walks a whole child's tree: child a (i = c + 1 + a) owns slots 0..a of a
// triangle, slot 0 for the child itself (its closed value, or phi(v, c) when
// it expands) and slot s >= 1 for its own child (floor(v / p_{c+s}), c+s-1),
// taken with the opposite sign when the child expands.
__global__ __launch_bounds__(SEED_T) void k_seed_rec(seed_ctx S, uint64_t m, uint32_t nb,
                                                     int64_t *term)
{
    __shared__ int64_t scr[SEED_T / 64];
    const uint32_t j = blockIdx.x + 1;
    if (j > nb)
        return;
    const uint32_t b = S.c + j;
    const uint64_t p = S.primes[b];
    const uint64_t u = pc_div(m, p, S.recip[b]);
    if (u < p * p) // closed (uniform over the workgroup)
        return;
    const uint64_t na = b - 1 - S.c, nslot = na * (na + 1) / 2;
    int64_t s = 0;
    for (uint64_t t = threadIdx.x; t < nslot; t += SEED_T) {
        // the child a with a (a + 1) / 2 <= t < (a + 1) (a + 2) / 2
        uint64_t a = (uint64_t)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((a + 1) * (a + 2) / 2 <= t)
            a++;
        while (a * (a + 1) / 2 > t)
            a--;
        const uint32_t slot = (uint32_t)(t - a * (a + 1) / 2);
        const uint32_t i = S.c + 1 + (uint32_t)a;
        const uint64_t v = pc_div(u, S.primes[i], S.recip[i]);
        int64_t lv;
        const bool closed = seed_leaf(S, v, i - 1, &lv);
        if (slot == 0) {
            s += closed ? lv : seed_wheel(S, v);
        } else if (!closed) {
            const uint32_t i2 = S.c + slot; // c < i2 < i
            s -= seed_phi(S, pc_div(v, S.primes[i2], S.recip[i2]), i2 - 1);
        }
    }
    s = pc_block_sum<SEED_T>(s, scr);
    if (threadIdx.x == 0)
        term[j] -= s;
}

// out[j] = term[0] - (term[1] + ... + term[j]) = phi(m, c + j), 0 <= j <= nb
__global__ __launch_bounds__(SCAN_T) void k_seed_scan(const int64_t *term, uint32_t nb,
                                                      uint64_t *out, int32_t *err)
{
    __shared__ int64_t scr[SCAN_T / 64];
    const uint32_t n = nb + 1, per = (n + SCAN_T - 1) / SCAN_T;
    const uint32_t j0 = threadIdx.x * per, j1 = min(n, j0 + per);
    int64_t loc = 0;
    for (uint32_t j = j0; j < j1; j++)
        loc += j ? -term[j] : term[j];
    int64_t tot;
    int64_t run = pc_block_excl_scan<SCAN_T>(loc, scr, &tot);
    bool neg = false;
    for (uint32_t j = j0; j < j1; j++) {
        run += j ? -term[j] : term[j];
        neg |= run < 0;
        out[j] = (uint64_t)run;
    }
    if (neg)
        atomicOr(err, 16);
}

} // namespace

hipError_t pc_launch_seed(const pc_tables &T, uint32_t c, uint64_t m, uint32_t nb,
                          uint32_t nrec, uint64_t pi_limit, int64_t *term, uint64_t *out,
                          int32_t *err, hipStream_t s)
{
    seed_ctx S{};
    S.primes = T.primes;
    S.recip = T.recip;
    S.pitab = T.pitab;
    S.phitab = T.phitab;
    S.pi_limit = pi_limit;
    S.Qc = T.Qc;
    S.rQc = pc_recip(T.Qc);
    S.phiQ = T.phiQ;
    S.c = c;
    S.err = err;
    k_seed_terms<<<(nb + SEED_T) / SEED_T, SEED_T, 0, s>>>(S, m, nb, term);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    nrec = std::min(nrec, nb);
    if (nrec) {
        k_seed_rec<<<nrec, SEED_T, 0, s>>>(S, m, nb, term);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    k_seed_scan<<<1, SCAN_T, 0, s>>>(term, nb, out, err);
    return hipGetLastError();
}

/*
 * oracle.c -- plain CPU reference for the combinatorial prime-counting method.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain, obviously-correct
 * reference ("oracle") that the GPU library is checked against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg load it.  The
 * library never links, calls or reads it, and the two share no source.
 *
 * Paper: D. B. Staple, "The combinatorial algorithm for computing pi(x)",
 * arXiv:1503.01839.  "§n", "eq. (4.1)" and "Table n" below refer to it.
 *
 * The paper names the pieces of the method but leaves their formulas to the
 * earlier literature (Lagarias-Miller-Odlyzko, Deleglise-Rivat, Oliveira e
 * Silva).  They are restated here from the mathematics:
 *
 *   phi(u,b)   #{1 <= n <= u : no p_i with i <= b divides n}          (§3)
 *   recurrence phi(u,b) = phi(u,b-1) - phi(floor(u/p_b), b-1)        (eq. (4.1))
 *   Meissel    pi(x) = phi(x,a) + a - 1 - P2(x,a),  a = pi(y),
 *              valid when p_{a+1}^3 > x (here y >= icbrt(x))          (§1, §4)
 *   P2(x,a)    #{n <= x : n = p*q, p_a < p <= q}
 *              = sum_{y < p <= sqrt x} (pi(x/p) - pi(p) + 1)
 *   Expanding eq. (4.1) from (1, a) and stopping at a node (n, b) once
 *   b = c (wheel size, §4) with n <= y, or once n > y, gives
 *     ordinary leaves  S1 = sum_{n <= y, mu(n) != 0, lpf(n) > p_c} mu(n) phi(x/n, c)
 *     special leaves   S2 = sum_{c < b < a} sum_{m in M_b} -mu(m) phi(x/(m p_b), b-1)
 *                      M_b = {m : mu(m) != 0, lpf(m) > p_b, y/p_b < m <= y}
 *   and phi(x,a) = S1 + S2.  With u = floor(x/(m p_b)) and p = p_b a special
 *   leaf is
 *     trivial  if u < p              (phi = 1),
 *     easy     if p <= u < p^2 and u <= y  (phi = pi(u) - b + 2, Legendre, §4),
 *     hard     otherwise             (phi read from a sieve of [1, x/y], §3).
 *
 * Every sum is exact integer arithmetic (signed 128-bit accumulators).
 * Floating point is used only inside the integer root helpers, whose result is
 * always corrected with exact integer comparisons.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

typedef struct {
    uint64_t lo;
    int64_t hi;
} or_i128;

static or_i128 pack(i128 v)
{
    or_i128 r;
    r.lo = (uint64_t)v;
    r.hi = (int64_t)(v >> 64);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Integer roots: floor(n^(1/2)) and floor(n^(1/3)), exact.                  */
/* ------------------------------------------------------------------------ */

uint64_t or_isqrt(uint64_t n)
{
    uint64_t r = (uint64_t)sqrtl((long double)n);
    while (r > 0 && (u128)r * r > n)
        r--;
    while ((u128)(r + 1) * (r + 1) <= n)
        r++;
    return r;
}

uint64_t or_icbrt(uint64_t n)
{
    uint64_t r = (uint64_t)cbrtl((long double)n);
    while (r > 0 && (u128)r * r * r > n)
        r--;
    while ((u128)(r + 1) * (r + 1) * (r + 1) <= n)
        r++;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Sieve of Eratosthenes (§1): primes up to a limit, and brute-force pi(n).  */
/* One byte per integer, segment by segment; nothing clever.                 */
/* ------------------------------------------------------------------------ */

#define OR_SEG (1u << 20)

/* primes <= limit, limit small enough for one byte array (<= ~1e9). */
static uint32_t *small_primes(uint64_t limit, uint64_t *count)
{
    unsigned char *comp = calloc(limit + 1, 1);
    uint64_t n = 0, cap = 1024;
    uint32_t *p = malloc(cap * sizeof *p);
    for (uint64_t i = 2; i <= limit; i++) {
        if (comp[i])
            continue;
        if (n == cap) {
            cap *= 2;
            p = realloc(p, cap * sizeof *p);
        }
        p[n++] = (uint32_t)i;
        for (uint64_t j = i * i; j <= limit; j += i)
            comp[j] = 1;
    }
    free(comp);
    *count = n;
    return p;
}

/* Walk the integers [0, hi] in segments; for every prime q met, in increasing
 * order, call visit(q, ctx).  Base primes up to sqrt(hi) cross the segments. */
typedef void (*prime_visitor)(uint64_t q, void *ctx);

static void for_each_prime(uint64_t hi, prime_visitor visit, void *ctx)
{
    uint64_t r = or_isqrt(hi), nb;
    uint32_t *base = small_primes(r, &nb);
    unsigned char *seg = malloc(OR_SEG);
    for (uint64_t lo = 0; lo <= hi; lo += OR_SEG) {
        uint64_t top = lo + OR_SEG - 1 > hi ? hi : lo + OR_SEG - 1;
        uint64_t len = top - lo + 1;
        memset(seg, 1, len);
        for (uint64_t i = 0; i < nb; i++) {
            uint64_t p = base[i];
            uint64_t start = p * p;
            if (start > top)
                break;
            if (start < lo)
                start = (lo + p - 1) / p * p;
            for (uint64_t j = start; j <= top; j += p)
                seg[j - lo] = 0;
        }
        for (uint64_t j = 0; j < len; j++)
            if (seg[j] && lo + j >= 2)
                visit(lo + j, ctx);
    }
    free(seg);
    free(base);
}

static void count_visit(uint64_t q, void *ctx)
{
    (void)q;
    (*(uint64_t *)ctx)++;
}

/* pi(n) by counting every prime <= n (§1, the sieve of Eratosthenes). */
uint64_t or_pi_brute(uint64_t n)
{
    uint64_t cnt = 0;
    if (n < 2)
        return 0;
    for_each_prime(n, count_visit, &cnt);
    return cnt;
}

typedef struct {
    uint32_t *p;
    uint64_t n, cap;
} prime_list;

static void list_visit(uint64_t q, void *ctx)
{
    prime_list *L = ctx;
    if (L->n < L->cap)
        L->p[L->n] = (uint32_t)q;
    L->n++;
}

/* Fill out[0..cap) with the primes <= n in order; return how many exist. */
uint64_t or_primes(uint64_t n, uint32_t *out, uint64_t cap)
{
    prime_list L = {out, 0, cap};
    if (n >= 2)
        for_each_prime(n, list_visit, &L);
    return L.n;
}

/* ------------------------------------------------------------------------ */
/* Shared context: primes, pi table, mu and lpf tables for one (x, y).       */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t x, y, a, c;
    uint32_t *p;      /* p[1..np] = primes <= plim; p[0] unused */
    uint64_t np, plim;
    uint32_t *pi;     /* pi[0..pilim] */
    uint64_t pilim;
    int8_t *mu;       /* mu[0..y]   */
    uint32_t *lpf;    /* lpf[0..y], lpf[1] = 0 meaning "no prime factor" */
} ctx_t;

static void ctx_free(ctx_t *C)
{
    free(C->p);
    free(C->pi);
    free(C->mu);
    free(C->lpf);
    memset(C, 0, sizeof *C);
}

/* Tables: primes and pi(.) up to pilim, mu and lpf up to y (§2.1, §2.2 name
 * these tables; the oracle simply stores them in full). */
static int ctx_init(ctx_t *C, uint64_t x, uint64_t y, uint64_t pilim)
{
    memset(C, 0, sizeof *C);
    C->x = x;
    C->y = y;
    if (pilim < y)
        pilim = y;
    if (pilim < 2)
        pilim = 2;
    C->pilim = pilim;
    uint64_t np;
    uint32_t *pr = small_primes(pilim, &np);
    C->np = np;
    C->plim = pilim;
    C->p = malloc((np + 2) * sizeof *C->p);
    C->p[0] = 0;
    memcpy(C->p + 1, pr, np * sizeof *pr);
    free(pr);
    C->pi = malloc((pilim + 1) * sizeof *C->pi);
    {
        uint64_t k = 0;
        for (uint64_t n = 0; n <= pilim; n++) {
            while (k < np && C->p[k + 1] <= n)
                k++;
            C->pi[n] = (uint32_t)k;
        }
    }
    C->a = C->pi[y];
    /* mu and least prime factor by a plain factor sieve */
    C->mu = malloc(y + 1);
    C->lpf = calloc(y + 1, sizeof *C->lpf);
    for (uint64_t n = 0; n <= y; n++)
        C->mu[n] = 1;
    for (uint64_t i = 1; i <= np && C->p[i] <= y; i++) {
        uint64_t q = C->p[i];
        for (uint64_t k = q; k <= y; k += q) {
            if (C->lpf[k] == 0)
                C->lpf[k] = (uint32_t)q;
            C->mu[k] = (int8_t)-C->mu[k];
        }
        if (q * q <= y)
            for (uint64_t k = q * q; k <= y; k += q * q)
                C->mu[k] = 0;
    }
    return 0;
}

/* mu(n) and the least prime factor lpf(n) for 0 <= n <= N (§2.2 keeps the
 * product mu(n) lpf(n) as a table), from the same plain factor sieve as the
 * context above: mu_out[n] in {-1, 0, 1}, lpf_out[n] the least prime factor
 * (0 for n < 2).  Returns 0, or -1 if N is too large for one byte array. */
int or_mu_lpf(uint64_t N, int8_t *mu_out, uint32_t *lpf_out)
{
    if (N > (1ull << 32))
        return -1;
    ctx_t C;
    ctx_init(&C, N, N < 2 ? 2 : N, 0);
    for (uint64_t n = 0; n <= N; n++) {
        mu_out[n] = n == 0 ? 0 : C.mu[n];
        lpf_out[n] = n < 2 ? 0 : C.lpf[n];
    }
    ctx_free(&C);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* phi(u, b)                                                                 */
/* ------------------------------------------------------------------------ */

/* Legendre's inclusion-exclusion for small b: sum over squarefree d | p_1..p_b
 * of mu(d) floor(u/d).  This is the wheel of size c (§4): phi(u,c) in O(1). */
static i128 phi_wheel(const ctx_t *C, uint64_t u, uint64_t b)
{
    i128 s = 0;
    for (uint64_t mask = 0; mask < (1ull << b); mask++) {
        u128 d = 1;
        int sign = 1;
        for (uint64_t i = 0; i < b; i++)
            if (mask >> i & 1) {
                d *= C->p[i + 1];
                sign = -sign;
            }
        if (d <= u)
            s += sign * (i128)(u / (uint64_t)d);
    }
    return s;
}

static uint64_t phi_nodes;

/* The recurrence eq. (4.1), with the shortcuts of §4:
 *   b <= c             : wheel;
 *   u < p_{b+1}        : only 1 survives, phi = 1;
 *   u < p_{b+1}^2, u in the pi table : Legendre, phi = pi(u) - b + 1. */
static i128 phi_rec(const ctx_t *C, uint64_t u, uint64_t b)
{
    phi_nodes++;
    if (u == 0)
        return 0;
    if (b == 0)
        return u;
    if (b <= C->c)
        return phi_wheel(C, u, b);
    if (b + 1 <= C->np) {
        uint64_t q = C->p[b + 1];
        if (u < q)
            return 1;
        if ((u128)u < (u128)q * q && u <= C->pilim)
            return (i128)C->pi[u] - (i128)b + 1;
    }
    return phi_rec(C, u, b - 1) - phi_rec(C, u / C->p[b], b - 1);
}

/* phi(u, b) for one (u, b).  The pi table reaches max(y, sqrt u). */
or_i128 or_phi(uint64_t u, uint64_t b, uint64_t c, uint64_t *nodes)
{
    ctx_t C;
    uint64_t lim = or_isqrt(u) + 2;
    if (lim < 1000)
        lim = 1000;
    ctx_init(&C, u, 2, lim);
    while (C.np < b + 1) { /* grow until p_{b+1} exists */
        uint64_t nl = C.pilim * 2;
        ctx_free(&C);
        ctx_init(&C, u, 2, nl);
    }
    C.c = c < b ? c : b;
    phi_nodes = 0;
    i128 r = phi_rec(&C, u, b);
    if (nodes)
        *nodes = phi_nodes;
    ctx_free(&C);
    return pack(r);
}

/* phi(u, b) by direct count: test each n <= u against p_1..p_b. */
uint64_t or_phi_direct(uint64_t u, uint64_t b)
{
    uint64_t np;
    uint32_t *pr = small_primes(64 + 20 * (b + 1) * 16, &np);
    uint64_t cnt = 0;
    for (uint64_t n = 1; n <= u; n++) {
        int ok = 1;
        for (uint64_t i = 0; i < b && i < np; i++)
            if (n % pr[i] == 0) {
                ok = 0;
                break;
            }
        cnt += ok;
    }
    free(pr);
    return cnt;
}

/* phi(m, b) for every 0 <= b <= b_hi at one m, straight from the definition
 * (§3): start from the integers 1..m and, for b = 1, 2, ..., remove the ones
 * that p_b divides and that are still present; out[b] is the number left.
 * This is the value a sieve started at m = m_min needs in every column
 * (§4, the seeding of phi(m_min, b)).  One byte per integer up to m.
 * Returns 0, or -1 if memory runs out. */
int or_phi_column(uint64_t m, uint64_t b_hi, uint64_t *out)
{
    uint64_t np = 0, lim = 64;
    uint32_t *pr;
    for (;;) {
        pr = small_primes(lim, &np);
        if (np >= b_hi)
            break;
        free(pr);
        lim *= 2;
    }
    unsigned char *gone = calloc(m + 1, 1);
    if (!gone) {
        free(pr);
        return -1;
    }
    uint64_t left = m;
    out[0] = m;
    for (uint64_t b = 1; b <= b_hi; b++) {
        const uint64_t p = pr[b - 1];
        for (uint64_t n = p; n <= m; n += p)
            if (!gone[n]) {
                gone[n] = 1;
                left--;
            }
        out[b] = left;
    }
    free(gone);
    free(pr);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* S1: ordinary leaves, enumerated with the nested loops of §2.2.            */
/* ------------------------------------------------------------------------ */

typedef struct {
    const ctx_t *C;
    i128 sum;
    uint64_t terms;
} s1_acc;

/* n is a squarefree product of primes with indices < i, all > p_c; sign = mu(n).
 * Each level of recursion is one more nested loop of §2.2. */
static void s1_loops(s1_acc *A, uint64_t n, uint64_t i, int sign)
{
    const ctx_t *C = A->C;
    A->sum += sign * phi_wheel(C, C->x / n, C->c);
    A->terms++;
    for (uint64_t j = i; j <= C->np && (u128)n * C->p[j] <= C->y; j++)
        s1_loops(A, n * C->p[j], j + 1, -sign);
}

/* ------------------------------------------------------------------------ */
/* P2 and pi at many points, by sieving [0, hi] once.                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    const uint64_t *q; /* ascending query points */
    uint64_t nq, k, cnt;
    uint64_t *out;     /* out[k] = pi(q[k]) */
} pi_at;

static void pi_at_visit(uint64_t p, void *ctx)
{
    pi_at *S = ctx;
    while (S->k < S->nq && S->q[S->k] < p)
        S->out[S->k++] = S->cnt;
    S->cnt++;
}

/* out[k] = pi(q[k]) for ascending q[] */
static void pi_at_points(const uint64_t *q, uint64_t nq, uint64_t *out)
{
    if (nq == 0)
        return;
    pi_at S = {q, nq, 0, 0, out};
    if (q[nq - 1] >= 2)
        for_each_prime(q[nq - 1], pi_at_visit, &S);
    while (S.k < nq)
        out[S.k++] = S.cnt;
}

/* P2(x, pi(y)) = sum over primes y < p <= sqrt x of (pi(x/p) - pi(p) + 1).
 * pi(x/p) for every p comes from one sieve of [0, x/(y+1)]. */
static i128 p2_sum(const ctx_t *C, uint64_t *nterms)
{
    uint64_t x = C->x, y = C->y, r = or_isqrt(x);
    uint64_t nsp;
    uint32_t *sp = small_primes(r, &nsp);
    uint64_t first = 0;
    while (first < nsp && sp[first] <= y)
        first++;
    uint64_t nq = nsp - first;
    uint64_t *q = malloc((nq + 1) * sizeof *q), *pq = malloc((nq + 1) * sizeof *pq);
    for (uint64_t k = 0; k < nq; k++) /* p descending -> x/p ascending */
        q[k] = x / sp[nsp - 1 - k];
    pi_at_points(q, nq, pq);
    i128 s = 0;
    for (uint64_t k = 0; k < nq; k++) {
        uint64_t idx = nsp - 1 - k;      /* p = sp[idx] is the (idx+1)-th prime */
        s += (i128)pq[k] - (i128)(idx + 1) + 1;
    }
    free(q);
    free(pq);
    free(sp);
    *nterms = nq;
    return s;
}

or_i128 or_p2(uint64_t x, uint64_t y)
{
    ctx_t C;
    memset(&C, 0, sizeof C);
    C.x = x;
    C.y = y;
    uint64_t n;
    return pack(p2_sum(&C, &n));
}

/* P2 by brute force for small x: count every n <= x that has exactly two
 * prime factors (with multiplicity), both larger than y. */
uint64_t or_p2_brute(uint64_t x, uint64_t y)
{
    uint64_t cnt = 0;
    for (uint64_t n = 4; n <= x; n++) {
        uint64_t m = n, k = 0, smallest = 0;
        for (uint64_t d = 2; d * d <= m; d++)
            while (m % d == 0) {
                if (!smallest)
                    smallest = d;
                m /= d;
                k++;
            }
        if (m > 1) {
            if (!smallest)
                smallest = m;
            k++;
        }
        if (k == 2 && smallest > y)
            cnt++;
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Special leaves.                                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t u;
    uint32_t b;
    int32_t w; /* -mu(m) */
} hard_leaf;

typedef struct {
    hard_leaf *v;
    uint64_t n, cap;
} leaf_vec;

static void leaf_push(leaf_vec *L, uint64_t u, uint32_t b, int32_t w)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1 << 16;
        L->v = realloc(L->v, L->cap * sizeof *L->v);
    }
    L->v[L->n].u = u;
    L->v[L->n].b = b;
    L->v[L->n].w = w;
    L->n++;
}

typedef struct {
    i128 s2t, s2e;
    uint64_t nt, ne, nh;
    leaf_vec hard; /* filled only when collecting */
    i128 *per_b_t, *per_b_e; /* optional, indexed by b */
    uint64_t u_max;          /* hard leaves with u > u_max are skipped (sampling only) */
} leaves_acc;

/* One special leaf (b, m): -mu(m) phi(x/(m p_b), b-1). */
static void one_leaf(const ctx_t *C, leaves_acc *A, uint64_t b, uint64_t m,
                     int mu_m, int collect)
{
    uint64_t p = C->p[b];
    uint64_t u = (uint64_t)(C->x / ((u128)m * p));
    int32_t w = -mu_m;
    if (u < p) { /* trivial: phi(u, b-1) = 1 */
        A->s2t += w;
        A->nt++;
        if (A->per_b_t)
            A->per_b_t[b] += w;
    } else if ((u128)u < (u128)p * p && u <= C->y) { /* easy: Legendre */
        i128 v = (i128)C->pi[u] - (i128)b + 2;
        A->s2e += w * v;
        A->ne++;
        if (A->per_b_e)
            A->per_b_e[b] += w * v;
    } else { /* hard */
        if (u > A->u_max)
            return;
        A->nh++;
        if (collect)
            leaf_push(&A->hard, u, (uint32_t)b, w);
    }
}

/* Enumerate every special leaf of M_b for c < b < a.  For p_b^2 <= y the
 * candidates m in (y/p_b, y] are tested against the mu and lpf tables.  For
 * p_b^2 > y every member of M_b is prime (m <= y < p_b^2 and lpf(m) > p_b), so
 * the primes in (max(p_b, y/p_b), y] are walked; the trailing run of them with
 * u < p_b is trivial and is counted, not walked. */
static void special_leaves(const ctx_t *C, leaves_acc *A, int collect, uint64_t b_lo,
                           uint64_t b_hi, uint64_t b_step)
{
    uint64_t x = C->x, y = C->y;
    if (b_step == 0)
        b_step = 1;
    while (b_lo < C->c + 1)
        b_lo += b_step;
    if (b_hi > C->a)
        b_hi = C->a;
    for (uint64_t b = b_lo; b < b_hi; b += b_step) {
        uint64_t p = C->p[b];
        uint64_t mlo = y / p + 1;
        if ((u128)p * p <= y) {
            for (uint64_t m = mlo; m <= y; m++)
                if (C->mu[m] != 0 && C->lpf[m] > p)
                    one_leaf(C, A, b, m, C->mu[m], collect);
        } else {
            /* trivial iff u < p iff m > x / p^2 */
            uint64_t tcut = (uint64_t)(x / ((u128)p * p));
            uint64_t jlo = C->pi[mlo > p + 1 ? mlo - 1 : p] + 1; /* first prime > max(p, mlo-1) */
            uint64_t jhi = C->a;                                  /* primes <= y */
            uint64_t jt = tcut >= y ? jhi + 1 : C->pi[tcut] + 1;  /* first trivial index */
            if (jt < jlo)
                jt = jlo;
            for (uint64_t j = jlo; j < jt && j <= jhi; j++)
                one_leaf(C, A, b, C->p[j], -1, collect);
            if (jt <= jhi) {
                uint64_t n = jhi - jt + 1; /* each contributes -mu(m) * 1 = +1 */
                A->s2t += (i128)n;
                A->nt += n;
                if (A->per_b_t)
                    A->per_b_t[b] += (i128)n;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Hard leaves by a direct segmented sieve of [1, z] with running counts     */
/* (the counters of §2.3, here a Fenwick tree per segment) and per-prime      */
/* carries phi(lo-1, b) between segments (§3, §4).                            */
/* ------------------------------------------------------------------------ */

static uint64_t hard_direct_unplaced;

static int leaf_cmp(const void *A, const void *B)
{
    const hard_leaf *a = A, *b = B;
    if (a->u != b->u)
        return a->u < b->u ? -1 : 1;
    return (a->b > b->b) - (a->b < b->b);
}

typedef struct {
    uint64_t lo;
    uint32_t *t; /* Fenwick tree, 1-based */
    uint64_t n;
} fenwick;

static void fw_add(fenwick *F, uint64_t i, int32_t d)
{
    for (i++; i <= F->n; i += i & (0 - i))
        F->t[i] += (uint32_t)d;
}

static uint64_t fw_sum(const fenwick *F, uint64_t i) /* sum of positions [0, i] */
{
    uint64_t s = 0;
    for (i++; i > 0; i -= i & (0 - i))
        s += F->t[i];
    return s;
}

/* Sum of -mu(m) phi(u, b-1) over the hard leaves.  per_b[b] (optional)
 * receives the per-prime sums, per_seg[s] (optional) the per-segment sums. */
static i128 hard_direct(const ctx_t *C, leaf_vec *L, uint64_t seglen, uint64_t bmax,
                        uint64_t z, i128 *per_b, i128 *per_seg, uint64_t nseg_cap)
{
    qsort(L->v, L->n, sizeof *L->v, leaf_cmp);
    /* leaves are now ascending in u; within one segment they are regrouped by b */
    unsigned char *flag = malloc(seglen);
    fenwick F;
    F.n = seglen;
    F.t = malloc((seglen + 1) * sizeof *F.t);
    uint64_t *carry = calloc(bmax + 2, sizeof *carry); /* carry[b] = phi(lo-1, b-1) */
    hard_leaf *buf = malloc((L->n + 1) * sizeof *buf);
    i128 total = 0;
    uint64_t li = 0;
    for (uint64_t lo = 0, s = 0; lo <= z; lo += seglen, s++) {
        uint64_t hi = lo + seglen; /* segment [lo, hi) */
        /* this segment's leaves, regrouped by b (stable within b) */
        uint64_t l0 = li;
        while (li < L->n && L->v[li].u < hi)
            li++;
        uint64_t nl = li - l0;
        {
            /* counting sort by b */
            uint64_t *cntb = calloc(bmax + 2, sizeof *cntb);
            for (uint64_t k = l0; k < li; k++)
                cntb[L->v[k].b]++;
            uint64_t acc = 0;
            for (uint64_t b = 0; b <= bmax + 1; b++) {
                uint64_t t = cntb[b];
                cntb[b] = acc;
                acc += t;
            }
            for (uint64_t k = l0; k < li; k++)
                buf[cntb[L->v[k].b]++] = L->v[k];
            free(cntb);
        }
        for (uint64_t i = 0; i < seglen; i++)
            flag[i] = (lo + i >= 1); /* n = 0 is not counted */
        memset(F.t, 0, (seglen + 1) * sizeof *F.t);
        for (uint64_t i = 0; i < seglen; i++)
            if (flag[i])
                fw_add(&F, i, 1);
        uint64_t alive = lo == 0 ? seglen - 1 : seglen;
        uint64_t k = 0;
        for (uint64_t b = 1; b <= bmax; b++) {
            /* leaves of b read phi(u, b-1): p_1..p_{b-1} are crossed */
            for (; k < nl && buf[k].b == b; k++) {
                uint64_t phi = carry[b] + fw_sum(&F, buf[k].u - lo);
                i128 t = (i128)buf[k].w * (i128)phi;
                total += t;
                if (per_b)
                    per_b[b] += t;
                if (per_seg && s < nseg_cap)
                    per_seg[s] += t;
            }
            carry[b] += alive;
            /* cross p_b and every multiple of it (phi semantics: p_b itself too) */
            uint64_t p = C->p[b];
            uint64_t first = (lo + p - 1) / p * p;
            if (first == 0)
                first = p;
            for (uint64_t n = first; n < hi; n += p)
                if (flag[n - lo]) {
                    flag[n - lo] = 0;
                    fw_add(&F, n - lo, -1);
                    alive--;
                }
        }
        if (k != nl)
            hard_direct_unplaced += nl - k; /* a hard leaf with b > bmax */
    }
    free(buf);
    free(carry);
    free(F.t);
    free(flag);
    return total;
}

/* ------------------------------------------------------------------------ */
/* The full decomposition                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t x, y, a, c, z, bmax;
    or_i128 s1, s2t, s2e, s2h, p2, phi;
    uint64_t n_s1, n_trivial, n_easy, n_hard, n_p2;
    uint64_t phi_nodes;
} or_decomp;

/* hard_route: 0 = S2h not computed;
 *             1 = S2h by the direct segmented sieve (hard_direct);
 *             2 = S2h = phi(x,a) - S1 - S2t - S2e, phi(x,a) by eq. (4.1);
 *             3 = both 1 and 2; s2h from the sieve, phi from the recursion.
 * want_phi: compute phi(x, a) by the recursion (implied by routes 2 and 3).
 * want_p2 : compute P2.
 * per_b_h / per_b_t / per_b_e (optional, length a+1): per-prime sums.
 * per_seg / nseg_cap (optional): per-segment hard sums, segments of seglen. */
int or_decompose(uint64_t x, uint64_t y, uint64_t c, int hard_route, int want_phi,
                 int want_p2, uint64_t seglen, or_decomp *out, or_i128 *per_b_h,
                 or_i128 *per_b_t, or_i128 *per_b_e, or_i128 *per_seg,
                 uint64_t nseg_cap)
{
    if (y < 1 || (u128)y * y > x || (u128)(y + 1) * (y + 1) * (y + 1) <= x)
        return 1; /* need icbrt(x) <= y <= isqrt(x) */
    ctx_t C;
    uint64_t z = x / y;
    uint64_t pilim = or_isqrt(x) + 1; /* pi(u) for the Legendre shortcut */
    if (pilim > (1ull << 27))
        pilim = 1ull << 27;
    if (pilim < or_isqrt(z) + 2)
        pilim = or_isqrt(z) + 2;
    ctx_init(&C, x, y, pilim);
    C.c = c < C.a ? c : C.a;
    memset(out, 0, sizeof *out);
    out->x = x;
    out->y = y;
    out->a = C.a;
    out->c = C.c;
    out->z = z;
    out->bmax = C.pi[or_isqrt(z)];
    if (seglen == 0)
        seglen = 1u << 20;

    /* S1 */
    s1_acc S = {&C, 0, 0};
    s1_loops(&S, 1, C.c + 1, 1);
    out->s1 = pack(S.sum);
    out->n_s1 = S.terms;

    /* special leaves */
    uint64_t nb = C.a + 1;
    i128 *pbt = per_b_t ? calloc(nb, sizeof(i128)) : NULL;
    i128 *pbe = per_b_e ? calloc(nb, sizeof(i128)) : NULL;
    leaves_acc A;
    memset(&A, 0, sizeof A);
    A.per_b_t = pbt;
    A.per_b_e = pbe;
    A.u_max = UINT64_MAX;
    int collect = hard_route == 1 || hard_route == 3;
    special_leaves(&C, &A, collect, C.c + 1, C.a, 1);
    out->s2t = pack(A.s2t);
    out->s2e = pack(A.s2e);
    out->n_trivial = A.nt;
    out->n_easy = A.ne;
    out->n_hard = A.nh;

    i128 s2h = 0, phi = 0;
    if (collect) {
        i128 *pbh = per_b_h ? calloc(nb, sizeof(i128)) : NULL;
        i128 *psg = per_seg ? calloc(nseg_cap, sizeof(i128)) : NULL;
        hard_direct_unplaced = 0;
        s2h = hard_direct(&C, &A.hard, seglen, out->bmax, z, pbh, psg, nseg_cap);
        if (hard_direct_unplaced) {
            free(pbh);
            free(psg);
            free(A.hard.v);
            free(pbt);
            free(pbe);
            ctx_free(&C);
            return 2;
        }
        if (pbh) {
            for (uint64_t b = 0; b < nb; b++)
                per_b_h[b] = pack(pbh[b]);
            free(pbh);
        }
        if (psg) {
            for (uint64_t s = 0; s < nseg_cap; s++)
                per_seg[s] = pack(psg[s]);
            free(psg);
        }
    }
    free(A.hard.v);
    if (want_phi || hard_route == 2 || hard_route == 3) {
        phi_nodes = 0;
        phi = phi_rec(&C, x, C.a);
        out->phi = pack(phi);
        out->phi_nodes = phi_nodes;
        if (hard_route == 2)
            s2h = phi - S.sum - A.s2t - A.s2e;
    }
    out->s2h = pack(s2h);
    if (pbt) {
        for (uint64_t b = 0; b < nb; b++)
            per_b_t[b] = pack(pbt[b]);
        free(pbt);
    }
    if (pbe) {
        for (uint64_t b = 0; b < nb; b++)
            per_b_e[b] = pack(pbe[b]);
        free(pbe);
    }
    if (want_p2) {
        uint64_t n2;
        out->p2 = pack(p2_sum(&C, &n2));
        out->n_p2 = n2;
    }
    ctx_free(&C);
    return 0;
}

/* Only the ordinary leaves S1 and P2 of one (x, y, c), with their term
 * counts, by the same routines as or_decompose (the special leaves of a large
 * x are summed separately, slice by slice, with or_leaf_sample). */
int or_s1_p2(uint64_t x, uint64_t y, uint64_t c, or_decomp *out)
{
    if (y < 1 || (u128)y * y > x || (u128)(y + 1) * (y + 1) * (y + 1) <= x)
        return 1;
    ctx_t C;
    uint64_t z = x / y;
    uint64_t pilim = or_isqrt(z) + 2;
    ctx_init(&C, x, y, pilim);
    C.c = c < C.a ? c : C.a;
    memset(out, 0, sizeof *out);
    out->x = x;
    out->y = y;
    out->a = C.a;
    out->c = C.c;
    out->z = z;
    out->bmax = C.pi[or_isqrt(z)];
    s1_acc S = {&C, 0, 0};
    s1_loops(&S, 1, C.c + 1, 1);
    out->s1 = pack(S.sum);
    out->n_s1 = S.terms;
    uint64_t n2;
    out->p2 = pack(p2_sum(&C, &n2));
    out->n_p2 = n2;
    ctx_free(&C);
    return 0;
}

/* pi(x) by Meissel's identity: phi(x, a) by eq. (4.1) plus P2, y given
 * (icbrt(x) <= y <= isqrt(x)).  Small x (< 8) is counted directly. */
uint64_t or_pi_meissel(uint64_t x, uint64_t y, uint64_t c)
{
    if (x < 8)
        return or_pi_brute(x);
    or_decomp D;
    if (or_decompose(x, y, c, 0, 1, 1, 0, &D, NULL, NULL, NULL, NULL, 0))
        return UINT64_MAX;
    i128 phi = ((i128)D.phi.hi << 64) | D.phi.lo;
    i128 p2 = ((i128)D.p2.hi << 64) | D.p2.lo;
    return (uint64_t)(phi + (i128)D.a - 1 - p2);
}

/* A bounded slice of the special leaves of one (x, y, c): the leaves with
 * b = b_lo + k b_step < b_hi (k >= 0; b_step 0 means 1; b <= c skipped), and
 * of the hard ones only those with u <= u_max (their phi from the direct
 * sieve of [1, u_max]).  Used to time the oracle on a sample of a workload
 * too large to run whole, and to sum a large one slice by slice.  out->n_*
 * count the leaves of the slice; out->s2t/s2e/s2h are the slice's sums. */
int or_leaf_sample(uint64_t x, uint64_t y, uint64_t c, uint64_t b_lo, uint64_t b_hi,
                   uint64_t b_step, uint64_t u_max, or_decomp *out)
{
    if (y < 1 || (u128)y * y > x || (u128)(y + 1) * (y + 1) * (y + 1) <= x)
        return 1;
    ctx_t C;
    ctx_init(&C, x, y, y + 2);
    C.c = c < C.a ? c : C.a;
    memset(out, 0, sizeof *out);
    out->x = x;
    out->y = y;
    out->a = C.a;
    out->c = C.c;
    out->z = x / y;
    leaves_acc A;
    memset(&A, 0, sizeof A);
    A.u_max = u_max;
    special_leaves(&C, &A, 1, b_lo, b_hi, b_step);
    out->s2t = pack(A.s2t);
    out->s2e = pack(A.s2e);
    out->n_trivial = A.nt;
    out->n_easy = A.ne;
    out->n_hard = A.nh;
    uint64_t bmax = b_hi > 0 ? b_hi - 1 : 0;
    if (bmax > C.a)
        bmax = C.a;
    out->bmax = bmax;
    hard_direct_unplaced = 0;
    i128 s2h = hard_direct(&C, &A.hard, 1u << 20, bmax, u_max, NULL, NULL, 0);
    out->s2h = pack(s2h);
    free(A.hard.v);
    ctx_free(&C);
    return hard_direct_unplaced ? 2 : 0;
}

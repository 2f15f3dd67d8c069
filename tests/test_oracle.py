"""Pins for the CPU oracle: it is checked against what the paper and plain
mathematics fix, never against itself.

* Table 1 and Table 2 of the paper (Section 5): exact pi(10^n), pi(2^m).
* Brute force on small inputs, written here in plain Python (trial division,
  gcd counts, factoring) and sharing nothing with oracle.c.
* Closed forms of phi (phi(u,1) = ceil(u/2), wheel periodicity, phi = 1 below
  p_{b+1}, phi(0,b) = 0).
* Invariants: phi(x,a) = S1 + S2 (Section 4's tree of eq. (4.1)); the two
  independent routes to the hard-leaf sum agree; pi(x) does not depend on
  alpha or on the wheel size c (the paper's own check, Section 5).
"""
import math
import random

import pytest

import oracle as O


# ---------------------------------------------------------------- helpers --
def is_prime(n):
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def py_primes(n):
    return [k for k in range(2, n + 1) if is_prime(k)]


def factor(n):
    f, d = [], 2
    while d * d <= n:
        while n % d == 0:
            f.append(d)
            n //= d
        d += 1
    if n > 1:
        f.append(n)
    return f


def mu(n):
    f = factor(n)
    return 0 if len(set(f)) != len(f) else (-1) ** len(f)


def lpf(n):
    return factor(n)[0] if n > 1 else math.inf


def phi_gcd(u, b, P):
    prod = 1
    for p in P[:b]:
        prod *= p
    return sum(1 for n in range(1, u + 1) if math.gcd(n, prod) == 1)


def brute_leaves(x, y, c):
    """Every special leaf by definition: (b, m), c < b < a, mu(m) != 0,
    lpf(m) > p_b, y < m p_b, m <= y; classified by u = x // (m p_b)."""
    P = py_primes(max(y, 50))
    a = sum(1 for p in P if p <= y)
    pi_tab = [0] * (y + 1)
    for n in range(2, y + 1):
        pi_tab[n] = pi_tab[n - 1] + is_prime(n)
    out = {"t": [0, 0], "e": [0, 0], "h": [0, 0]}
    for b in range(c + 1, a):
        p = P[b - 1]
        for m in range(1, y + 1):
            if m * p <= y or mu(m) == 0 or lpf(m) <= p:
                continue
            u = x // (m * p)
            w = -mu(m)
            if u < p:
                out["t"][0] += 1
                out["t"][1] += w
            elif u < p * p and u <= y:
                out["e"][0] += 1
                out["e"][1] += w * (pi_tab[u] - b + 2)
            else:
                out["h"][0] += 1
                out["h"][1] += w * phi_gcd(u, b - 1, P)
    return a, out


# ----------------------------------------------------------- the tables ----
def test_primes_and_roots_small():
    assert O.primes(10000) == py_primes(10000)
    for n in list(range(0, 3000)) + [2**63 - 1, 2**63, 2**64 - 1, 10**18, 10**18 - 1]:
        r = O.isqrt(n)
        assert r * r <= n < (r + 1) ** 2
        t = O.icbrt(n)
        assert t ** 3 <= n < (t + 1) ** 3


def test_pi_brute_vs_trial_division():
    count = 0
    for n in range(0, 5001):
        count += is_prime(n)
        if n % 7 == 0 or n < 200:
            assert O.pi_brute(n) == count, n


def test_pi_brute_paper_tables(paper_pow10, paper_pow2):
    # Table 1 (n <= 9) and Table 2 (m <= 30), Section 5
    for n in range(1, 10):
        assert O.pi_brute(10**n) == paper_pow10[n], n
    for m in range(1, 31):
        assert O.pi_brute(2**m) == paper_pow2[m], m


# ------------------------------------------------------------------ phi ----
def test_phi_recurrence_vs_gcd_count():
    P = py_primes(200)
    rng = random.Random(1503)
    for _ in range(120):
        u = rng.randrange(0, 3000)
        b = rng.randrange(0, 12)
        c = rng.choice([0, 1, 3, 6])
        want = phi_gcd(u, b, P)
        assert O.phi(u, b, c) == want, (u, b, c)
        assert O.phi_direct(u, b) == want, (u, b)


def test_phi_closed_forms():
    rng = random.Random(7)
    P = py_primes(1000)
    for _ in range(200):
        u = rng.randrange(0, 10**7)
        assert O.phi(u, 1, 1) == (u + 1) // 2
        assert O.phi(u + 30030, 6, 6) == O.phi(u, 6, 6) + 5760
        assert O.phi(u + 30030, 6, 0) == O.phi(u, 6, 0) + 5760
    for b in range(0, 40):
        assert O.phi(0, b) == 0
        for u in (1, P[b] - 1) if b < len(P) else ():
            if u >= 1 and b >= 1:
                assert O.phi(u, b) == 1
    # Legendre: p_b <= u < p_{b+1}^2  =>  phi(u, b) = pi(u) - b + 1
    for b in (5, 10, 30):
        for u in (P[b], P[b] ** 2 - 1, P[b] * P[b + 1] - 1):
            if u < P[b] ** 2:
                assert O.phi(u, b) == O.pi_brute(u) - b + 1


def test_phi_column_pins():
    # phi(m, b) for every b at one m (the seed of a sieve started at m, §4)
    P = py_primes(4000)
    rng = random.Random(41)
    for _ in range(40):  # gcd counts, written here
        m = rng.randrange(0, 2500)
        col = O.phi_column(m, 30)
        for b in range(31):
            assert int(col[b]) == phi_gcd(m, b, P), (m, b)
    for m in (1, 2, 3, 30030, 10**6 + 7, 3 * 10**6 + 1):
        n_pi = sum(1 for p in P if p <= m) if m <= P[-1] else None
        col = O.phi_column(m, 500)
        assert int(col[0]) == m and int(col[1]) == (m + 1) // 2
        if m >= 30030:
            assert int(O.phi_column(m + 30030, 6)[6]) == int(col[6]) + 5760
        if n_pi is not None:  # below p_{b+1}^2 and from pi(m) on: closed forms
            r = math.isqrt(m)
            for b in range(1, 501):
                if P[b - 1] <= r:
                    continue
                assert int(col[b]) == max(n_pi - b + 1, 1), (m, b)
    # the recurrence eq. (4.1) of the oracle, sampled at a larger m
    m = 12_345_679
    col = O.phi_column(m, 800)
    for b in (0, 6, 7, 8, 30, 100, 301, 446, 447, 800):
        assert int(col[b]) == O.phi(m, b), b
    # Legendre at m: pi(m) - b + 1 for pi(sqrt m) <= b, pi(m) from a plain sieve
    sv = bytearray([1]) * (m + 1)
    sv[0] = sv[1] = 0
    for q in range(2, math.isqrt(m) + 1):
        if sv[q]:
            sv[q * q::q] = bytearray(len(range(q * q, m + 1, q)))
    pm = sum(sv)
    kr = sum(1 for p in P if p * p <= m)
    for b in (kr, kr + 1, 600, 800):
        assert int(col[b]) == pm - b + 1, b


def test_phi_column_legendre_tail_vs_table1(paper_pow10):
    # past pi(sqrt m) the column is pi(m) - b + 1, pi(10^8) from Table 1
    m = 10**8
    kr = sum(1 for p in py_primes(10**4) if p * p <= m)  # pi(sqrt m) = pi(10^4)
    col = O.phi_column(m, kr + 40)
    for b in range(kr, kr + 41):
        assert int(col[b]) == paper_pow10[8] - b + 1, b
    assert int(col[6]) == 5760 * (m // 30030) + int(O.phi_column(m % 30030, 6)[6])


def test_phi_large_vs_meissel_and_table(paper_pow10):
    # phi(x, pi(icbrt x)) + a - 1 - P2 reproduces Table 1 for n <= 12
    for n in range(3, 13):
        x = 10**n
        assert O.pi_meissel(x) == paper_pow10[n], n


def test_meissel_powers_of_two(paper_pow2):
    for m in range(3, 37):
        assert O.pi_meissel(2**m) == paper_pow2[m], m


# ------------------------------------------------------------------- P2 ----
def test_p2_vs_semiprime_count():
    rng = random.Random(11)
    for x in [8, 27, 100, 1000, 12345, 30000] + [rng.randrange(8, 40000) for _ in range(6)]:
        lo, hi = O.icbrt(x), O.isqrt(x)
        for y in sorted({lo, (lo + hi) // 2, hi}):
            assert O.p2(x, y) == O.p2_brute(x, y), (x, y)
            # and by Python factoring
            want = sum(1 for n in range(4, x + 1)
                       if len(factor(n)) == 2 and factor(n)[0] > y)
            if x <= 12345:
                assert O.p2(x, y) == want, (x, y)


# --------------------------------------------------------- decomposition ---
@pytest.mark.parametrize("x,y", [(1000, 10), (1000, 31), (5000, 17), (5000, 40),
                                 (10**4, 21), (10**4, 60), (30030, 31), (40000, 100)])
@pytest.mark.parametrize("c", [0, 1, 2, 6])
def test_leaves_vs_definition(x, y, c):
    a, want = brute_leaves(x, y, c)
    cc = min(c, a)
    if cc != c:
        a, want = brute_leaves(x, y, cc)
    d = O.decompose(x, y, c, hard=O.HARD_BOTH, want_phi=True)
    assert d.a == a
    assert (d.n_trivial, d.s2t) == tuple(want["t"])
    assert (d.n_easy, d.s2e) == tuple(want["e"])
    assert (d.n_hard, d.s2h) == tuple(want["h"])
    P = py_primes(1000)
    assert d.phi == phi_gcd(x, a, P)
    assert d.s1 + d.s2t + d.s2e + d.s2h == d.phi
    assert d.pi == sum(1 for n in range(x + 1) if is_prime(n))


def test_s1_by_definition():
    P = py_primes(1000)
    for x, y, c in [(10**4, 21, 2), (10**5, 46, 6), (10**5, 100, 0), (99991, 300, 3)]:
        d = O.decompose(x, y, c, hard=O.HARD_NONE, want_p2=False)
        cc = d.c
        pc = P[cc - 1] if cc > 0 else 1
        s1 = sum(mu(n) * phi_gcd(x // n, cc, P) for n in range(1, y + 1)
                 if mu(n) != 0 and lpf(n) > pc)
        assert d.s1 == s1


def test_identity_routes_agree_random():
    rng = random.Random(1839)
    for _ in range(20):
        x = rng.randrange(10**4, 10**8)
        lo, hi = O.icbrt(x), O.isqrt(x)
        y = rng.choice([lo, min(hi, 2 * lo), min(hi, 8 * lo), hi])
        c = rng.choice([0, 1, 4, 6])
        d = O.decompose(x, y, c, hard=O.HARD_BOTH, want_phi=True, seglen=rng.choice([0, 4096, 65536]))
        assert d.s1 + d.s2t + d.s2e + d.s2h == d.phi, (x, y, c)
        assert d.pi == O.pi_brute(x), (x, y, c)


def test_pi_invariant_in_alpha_and_c(paper_pow10):
    # Section 5: values were recomputed with differing alpha, c and L.
    for n in (9, 10, 11):
        x = 10**n
        r = O.icbrt(x)
        for alpha in (1, 2, 4, 8):
            y = min(alpha * r, O.isqrt(x))
            for c in (0, 1, 6):
                d = O.decompose(x, y, c, hard=O.HARD_SIEVE, seglen=1 << 18)
                assert d.pi == paper_pow10[n], (n, alpha, c)


def test_per_b_sums_add_up():
    d = O.decompose(10**8, 464 * 2, 6, hard=O.HARD_SIEVE, per_b=True, nseg=64, seglen=1 << 16)
    assert sum(d.per_b_hard) == d.s2h
    assert sum(d.per_b_trivial) == d.s2t
    assert sum(d.per_b_easy) == d.s2e
    assert sum(d.per_seg_hard) == d.s2h


def test_survey_worked_values():
    # Values a separate throwaway computation produced; reproduced, not authority.
    d = O.decompose(10**6, 100, 1, hard=O.HARD_BOTH, want_phi=True)
    assert (d.phi, d.p2, d.s1, d.s2h, d.n_hard) == (120760, 42286, 24853, 95907, 269)
    d = O.decompose(10**6, 200, 6, hard=O.HARD_BOTH, want_phi=True)
    assert (d.phi, d.p2, d.s2t, d.s2e, d.s1, d.s2h) == (102753, 24300, 271, 4092, 75754, 22636)
    d = O.decompose(10**11, 4641, 6, hard=O.HARD_SIEVE)
    assert (d.s1, d.s2h, d.n_hard, d.p2, d.bmax) == (1469551610, 5219697028, 192435, 2571194450, 626)


# ------------------------------------------------ tables and leaf slices ---
def test_mu_lpf_vs_factoring():
    N = 20000
    m, l = O.mu_lpf(N)
    for n in range(N + 1):
        if n < 2:
            assert l[n] == 0 and m[n] == (1 if n == 1 else 0), n
            continue
        assert m[n] == mu(n), n
        assert l[n] == factor(n)[0], n


def test_leaf_sample_vs_per_b_sums():
    # a slice of b with every hard leaf (u_max = z) equals the per-prime sums
    # of the whole decomposition over the same b
    for x, y in [(10**8, 928), (10**9, 4000), (10**9 + 7, 31622)]:
        d = O.decompose(x, y, 6, hard=O.HARD_SIEVE, per_b=True)
        for b0, b1 in [(0, d.a), (7, 9), (10, 60), (d.a // 3, d.a // 2), (d.a - 5, d.a)]:
            s = O.leaf_sample(x, y, 6, b0, b1, d.z)
            lo = max(b0, 7)
            assert s.s2t == sum(d.per_b_trivial[lo:b1]), (x, y, b0, b1)
            assert s.s2e == sum(d.per_b_easy[lo:b1]), (x, y, b0, b1)
            assert s.s2h == sum(d.per_b_hard[lo:b1]), (x, y, b0, b1)
        s = O.leaf_sample(x, y, 6, 0, d.a, d.z)
        assert (s.n_trivial, s.n_easy, s.n_hard) == (d.n_trivial, d.n_easy, d.n_hard)
        # every b_step-th prime from b_lo on
        for b0, step in [(7, 5), (9, 64), (0, 3)]:
            s = O.leaf_sample(x, y, 6, b0, d.a, d.z, b_step=step)
            bs = [b for b in range(b0, d.a, step) if b >= 7]
            assert s.s2t == sum(d.per_b_trivial[b] for b in bs), (x, y, b0, step)
            assert s.s2e == sum(d.per_b_easy[b] for b in bs), (x, y, b0, step)
            assert s.s2h == sum(d.per_b_hard[b] for b in bs), (x, y, b0, step)


def test_leaf_sample_u_bound_vs_definition():
    # hard leaves only up to u_max: brute force by definition (gcd-count phi)
    P = py_primes(1000)
    for x, y, c, b0, b1, umax in [(10**4, 21, 2, 0, 99, 300), (40000, 100, 6, 7, 20, 2000),
                                  (30030, 31, 1, 2, 9, 500)]:
        s = O.leaf_sample(x, y, c, b0, b1, umax)
        a = sum(1 for p in P if p <= y)
        cc = min(c, a)
        nt = st = ne = se = nh = sh = 0
        pi_tab = [0] * (y + 1)
        for n in range(2, y + 1):
            pi_tab[n] = pi_tab[n - 1] + is_prime(n)
        for b in range(max(b0, cc + 1), min(b1, a)):
            p = P[b - 1]
            for m in range(1, y + 1):
                if m * p <= y or mu(m) == 0 or lpf(m) <= p:
                    continue
                u, w = x // (m * p), -mu(m)
                if u < p:
                    nt, st = nt + 1, st + w
                elif u < p * p and u <= y:
                    ne, se = ne + 1, se + w * (pi_tab[u] - b + 2)
                elif u <= umax:
                    nh, sh = nh + 1, sh + w * phi_gcd(u, b - 1, P)
        assert (s.n_trivial, s.s2t, s.n_easy, s.s2e, s.n_hard, s.s2h) == (nt, st, ne, se, nh, sh)


def test_s1_p2_vs_decompose():
    for x, y in [(10**9, 1000), (10**10 + 3, 9000), (2**36, 4096)]:
        d = O.decompose(x, y, 6, hard=O.HARD_NONE)
        e = O.s1_p2(x, y, 6)
        assert (e.s1, e.n_s1, e.p2, e.n_p2, e.a, e.bmax) == (d.s1, d.n_s1, d.p2, d.n_p2, d.a, d.bmax)


"""Windows of the sieve seeded on their own (Section 4): phi(m_min, b) for one
m_min and every b, from the wheel's phi(m, c) by eq. (4.1) with the closed
rules of Section 4 (pc_phi_seed), and whole queries whose windows take those
seeds instead of the carries of the windows before them (PC_FLAG_SEEDED, run
last to first).

Pins: the oracle's phi column (counted from the definition) at m up to
2 * 10^8; at m up to 2^46 Legendre's closed form past pi(sqrt m), phi(m, b) =
pi(m) - b + 1 with pi(m) from Tables 1 and 2, and the wheel's phi(m, 6) written
out here; seeded queries against the chained ones, the oracle and the tables.
"""
import math

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def wheel6(m):
    # phi(m, 6) over the primes 2 .. 13 by inclusion-exclusion, written here
    ps = [2, 3, 5, 7, 11, 13]
    s = 0
    for mask in range(64):
        d, k = 1, 0
        for i in range(6):
            if mask >> i & 1:
                d *= ps[i]
                k += 1
        s += (-1) ** k * (m // d)
    return s


@pytest.mark.parametrize("m,c,b_hi", [
    (0, 6, 40), (1, 6, 40), (2, 1, 30), (30029, 1, 200), (30030, 6, 200), (10**6 + 1, 6, 400),
    (2**24 - 1, 6, 1200), (123_456_789, 6, 3000), (99_999_999, 3, 2000),
    (200_000_003, 6, 2500), (7_777_777, 2, 900)])
def test_seeds_vs_oracle_column(pc, m, c, b_hi):
    say(f"case: seeds m={m} c={c} b_hi={b_hi}")
    got = pc.phi_seed(m, b_hi, c)
    want = O.phi_column(m, b_hi)[c:]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("src,k", [("pow10", 11), ("pow10", 12), ("pow10", 13),
                                   ("pow2", 40), ("pow2", 44), ("pow2", 46)])
def test_seeds_legendre_tail_vs_tables(pc, paper_pow10, paper_pow2, src, k):
    # past pi(sqrt m) every column is pi(m) - b + 1: the sum of all the terms
    # of eq. (4.1), expanded and closed ones, against the paper's pi(m)
    m = 10**k if src == "pow10" else 2**k
    pm = paper_pow10[k] if src == "pow10" else paper_pow2[k]
    r = math.isqrt(m)
    kr = int(pc.read_table(pc.TABLE_PI, r, 1)[0])  # pi(sqrt m)
    b_hi = kr + 64
    say(f"case: seeds m={src}^{k} b_hi={b_hi}")
    got = pc.phi_seed(m, b_hi, 6).astype(object)
    assert got[0] == wheel6(m)
    assert all(got[i] >= got[i + 1] for i in range(len(got) - 1))
    for b in range(kr, b_hi + 1):
        assert got[b - 6] == pm - b + 1, b


def test_seed_refusals(pc):
    out = np.zeros(8, dtype=np.uint64)
    L = pc.lib()
    assert L.pc_phi_seed(10, 0, 5, out.ctypes.data) == pc.PC_EINVAL
    assert L.pc_phi_seed(10, 7, 6, out.ctypes.data) == pc.PC_EINVAL
    assert L.pc_phi_seed(10, 6, 7, None) == pc.PC_EINVAL
    assert L.pc_phi_seed((1 << 48) + 1, 6, 7, out.ctypes.data) == pc.PC_ERANGE
    assert L.pc_phi_seed(10, 6, 1 << 27, out.ctypes.data) == pc.PC_ERANGE


def test_seeded_windows_vs_chained_and_oracle(pc):
    # tiny carry budgets: many windows, each seeded at its first integer
    for x, y in ((10**12, 10**4), (10**13, 40_000), (10**14 + 7, 100_000)):
        o = O.decompose(x, y, 6, hard=O.HARD_SIEVE)
        for budget in (1 << 13, 1 << 16):
            for two in (0, pc.FLAG_TWO_PASS):
                say(f"case: seeded x={x} y={y} budget={budget} two_pass={bool(two)}")
                r = pc.decompose(x, y, carry_budget=budget, flags=pc.FLAG_SEEDED | two)
                assert r.windows > 1
                assert (r.s2_hard, r.p2, r.pi) == (o.s2h, o.p2, o.pi), (x, y, budget, two)


def test_seeded_windows_large(pc, paper_pow10, paper_pow2):
    # at 1e18 the seeds reach m ~ z = 4e10 (hundreds of expanded columns)
    cases = [(10**16, paper_pow10[16], 1 << 22), (10**18, paper_pow10[18], 1 << 26),
             (2**62, paper_pow2[62], 1 << 27)]
    for x, want, budget in cases:
        say(f"case: seeded x={x} budget={budget}")
        r = pc.pi_count_ex(x, carry_budget=budget, flags=pc.FLAG_SEEDED)
        c = pc.pi_count_ex(x, carry_budget=budget)
        assert r.windows > 1 and r.windows == c.windows
        assert r.pi == want and c.pi == want
        assert (r.s2_hard, r.p2) == (c.s2_hard, c.p2)


def test_seeded_windows_wide(pc, paper_pow2):
    say("case: seeded 2^65")
    r = pc.pi_count_wide(2**65, carry_budget=1 << 28, flags=pc.FLAG_SEEDED)
    assert r.windows > 1
    assert r.pi == paper_pow2[65]


def test_seeded_windows_in_batches(pc, paper_pow10):
    # a batch whose large members run alone in seeded windows
    xs = [10**9, 10**13 + 1, 10**14, 3 * 10**11, 10**13]
    say("case: batch with seeded windows")
    solo = [pc.pi_count(x) for x in xs]
    for budget in (1 << 16, 1 << 20):
        assert pc.pi_count_batch(xs, carry_budget=budget, flags=pc.FLAG_SEEDED) == solo, budget
    assert solo[2] == paper_pow10[14] and solo[4] == paper_pow10[13]


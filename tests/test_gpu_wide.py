"""pi(x) above 2^64 (pc_pi_count_wide) against Tables 1 and 2 (Section 5).

Up to 2^72 every leaf quotient, every x / p of P2 and every segment bound
still fits 64 bits; X_b (128-bit below p_b < x / 2^64), S1's x / n, the
per-segment bounds of P2 and pi(x) itself (from 2^70 on) are formed in 128
bits.  The pi table then reaches isqrt(x) > 2^32, with the primes above 2^32
held as 64-bit values.
"""
import ctypes as C

import pytest

WIDE = [64, 65, 66, 67, 68, 69, 70, 71, 72]


def say(*a):
    print(*a, flush=True)


@pytest.mark.gpu
def test_last_u64_and_first_wide(pc, paper_pow2):
    # pi(2^64 - 1) = pi(2^64): the top of the 64-bit domain, both entry points
    say("step: pi(2^64 - 1) and pi(2^64)")
    assert pc.pi_count((1 << 64) - 1) == paper_pow2[64]
    r = pc.pi_count_wide(1 << 64)
    assert (r.x, r.x_hi, r.pi) == (1 << 64, 1, paper_pow2[64])
    assert r.phi == r.s1 + r.s2_trivial + r.s2_easy + r.s2_hard


@pytest.mark.gpu
@pytest.mark.parametrize("m", WIDE)
def test_table2_wide(pc, paper_pow2, m):
    say(f"step: pi(2^{m})")
    r = pc.pi_count_wide(1 << m)
    assert r.pi == paper_pow2[m]
    assert r.pi == r.phi + r.a - 1 - r.p2


@pytest.mark.gpu
@pytest.mark.parametrize("n", [20, 21])
def test_table1_wide(pc, paper_pow10, n):
    say(f"step: pi(10^{n})")
    r = pc.pi_count_wide(10**n)
    assert r.pi == paper_pow10[n]
    assert r.pi == r.phi + r.a - 1 - r.p2


@pytest.mark.gpu
def test_wide_alpha_invariance(pc, paper_pow2):
    # another y moves work between S1, the three leaf classes and P2; pi must not move
    x = (1 << 64) + (1 << 62)
    say("step: alpha invariance at 2^64 + 2^62")
    r1 = pc.pi_count_wide(x, alpha=12.0)
    r2 = pc.pi_count_wide(x, alpha=64.0)
    assert r1.y != r2.y and r1.s2_hard != r2.s2_hard and r1.p2 != r2.p2
    assert r1.pi == r2.pi
    assert paper_pow2[64] < r1.pi < paper_pow2[65]


@pytest.mark.gpu
def test_wide_matches_narrow_below_2_64(pc, paper_pow10):
    # the wide entry point on x < 2^64, after the tables grew past 2^32
    say("step: wide entry below 2^64")
    pc.pi_count_wide(1 << 65)
    for x in (10**12, 10**16, (1 << 63) + (1 << 61)):
        assert pc.pi_count_wide(x).pi == pc.pi_count(x)
    assert pc.pi_count(10**18) == paper_pow10[18]
    assert list(pc.read_table(pc.TABLE_PRIMES, 1, 5)) == [2, 3, 5, 7, 11]


@pytest.mark.gpu
def test_wide_range_refused(pc):
    r = pc._Result()
    for lo, hi in [(1, 256), (0, 257), ((1 << 64) - 1, (1 << 64) - 1)]:
        assert pc.lib().pc_pi_count_wide(lo, hi, None, C.byref(r)) == pc.PC_ERANGE
    with pytest.raises(ValueError):
        pc.pi_count_wide((1 << 72) + 1)

"""x at and above 2^63 (unsigned 64-bit quotients): Table 1's pi(10^19) and
Table 2's pi(2^63) through the GPU path, and 2^63 + 2^61, which the paper does
not tabulate (parity unpinned there): its pi(x) must not depend on alpha or on
the segment shape, and must lie between pi(2^63) and pi(2^64)."""
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_paper_values_above_2_63(pc, paper_pow10, paper_pow2):
    say("case: pi(2^63)")
    assert pc.pi_count(2**63) == paper_pow2[63]
    say("case: pi(10^19)")
    assert pc.pi_count(10**19) == paper_pow10[19]


def test_2_63_plus_2_61_invariance(pc, paper_pow2):
    x = 2**63 + 2**61
    vals = []
    for kw in (dict(alpha=8), dict(alpha=16), dict(alpha=4, tile_leaves=0xFFFFFFFF)):
        say("case: 2^63+2^61", kw)
        vals.append(pc.pi_count_ex(x, **kw).pi)
    assert len(set(vals)) == 1
    assert paper_pow2[63] < vals[0] < paper_pow2[64]

"""The shared device tables (Section 2.1's primes and pi(.), Section 2.2's
mu(n) * lpf(n)) read back through pc_read_table and compared entry by entry
with the CPU oracle's plain sieves.

The mu * lpf table is rebuilt several times at the size the headline query
uses (y = 3.6e7, pi(10^18) at alpha 36): every build must equal the oracle's,
since a table kernel whose threads race would differ from build to build.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

Y_HEADLINE = 36_000_000


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def oracle_mu_lpf():
    mu, lpf = O.mu_lpf(Y_HEADLINE)
    return mu, lpf


def expected_mulpf(mu, lpf, lo, n):
    """The library's encoding: mu(v) * lpf(v); 0 at v = 0 and for mu(v) = 0;
    INT32_MAX at v = 1 (no prime factor)."""
    m = mu[lo:lo + n].astype(np.int64)
    l = lpf[lo:lo + n].astype(np.int64)
    want = m * l
    if lo <= 1 < lo + n:
        want[1 - lo] = 2**31 - 1
    return want


def test_mulpf_every_build(pc, oracle_mu_lpf):
    mu, lpf = oracle_mu_lpf
    want = expected_mulpf(mu, lpf, 0, Y_HEADLINE + 1)
    for k in range(6):
        pc.shutdown()  # drop every table: the next read builds mu * lpf afresh
        say("case: mu*lpf build", k, "up to", Y_HEADLINE)
        got = pc.read_table(pc.TABLE_MULPF, 0, Y_HEADLINE + 1).astype(np.int64)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, f"build {k}: {bad.size} entries differ, first n = {bad[:8].tolist()}"


def test_mulpf_offset_ranges(pc, oracle_mu_lpf):
    mu, lpf = oracle_mu_lpf
    for lo, n in [(0, 1), (1, 5), (4095, 3), (19110979 - 7, 15), (Y_HEADLINE - 100, 101)]:
        say("case: mu*lpf range", lo, n)
        got = pc.read_table(pc.TABLE_MULPF, lo, n).astype(np.int64)
        assert (got == expected_mulpf(mu, lpf, lo, n)).all(), (lo, n)


def test_primes_and_pi(pc):
    N = 10**7
    ps = np.array(O.primes(N), dtype=np.uint32)
    say("case: primes", len(ps))
    got = pc.read_table(pc.TABLE_PRIMES, 1, len(ps))
    assert (got == ps).all()
    say("case: pi table to", N)
    pi = pc.read_table(pc.TABLE_PI, 0, N + 1)
    want = np.zeros(N + 1, dtype=np.uint64)
    want[ps] = 1
    want = np.cumsum(want)
    assert (pi == want).all()
    # the largest values the table holds: p_k and pi near 2^32 (Table 2: pi(2^32))
    top = pc.read_table(pc.TABLE_PI, 2**32 - 1, 1)
    assert int(top[0]) == 203280221


def test_read_table_rejects(pc):
    with pytest.raises(pc.PicountError):
        pc.read_table(pc.TABLE_PRIMES, 0, 4)       # primes are numbered from 1
    with pytest.raises(pc.PicountError):
        pc.read_table(pc.TABLE_MULPF, 2**31 - 2, 2)  # beyond the table's domain
    with pytest.raises(pc.PicountError):
        pc.read_table(pc.TABLE_PI, 2**32, 1)
    with pytest.raises(ValueError):
        pc.read_table(99, 0, 1)
    buf = np.zeros(1, dtype=np.uint64)
    assert pc.lib().pc_read_table(99, 0, 1, buf.ctypes.data) == pc.PC_EINVAL
    assert len(pc.read_table(pc.TABLE_PI, 5, 0)) == 0


def test_rebuild_in_place_sequence(pc, oracle_mu_lpf, paper_pow10, paper_pow2):
    # PC_FLAG_REBUILD_TABLES rebuilds every table into the device memory it
    # already holds: through a growing and a shrinking pi table (above 2^32 at
    # 2^65, with the primes past 2^32 as 64-bit values) each query still
    # returns the paper's pi, and the mu * lpf table read after the rebuilds
    # equals the oracle's
    mu, lpf = oracle_mu_lpf
    rb = pc.FLAG_REBUILD_TABLES
    seq = [(10**18, paper_pow10[18]), (10**12, paper_pow10[12]), (2**65, paper_pow2[65]),
           (10**15, paper_pow10[15]), (10**18, paper_pow10[18])]
    for x, want in seq:
        say("case: rebuild in place, x =", x)
        got = pc.pi_count_wide(x, flags=rb).pi if x >> 64 else pc.pi_count_ex(x, flags=rb).pi
        assert got == want, x
    got = pc.read_table(pc.TABLE_MULPF, 0, Y_HEADLINE + 1).astype(np.int64)
    assert (got == expected_mulpf(mu, lpf, 0, Y_HEADLINE + 1)).all()

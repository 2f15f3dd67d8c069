"""The library's pi table (a bitmap with a prefix count per 64 integers, one
read per lookup) against the sampled table of the paper's Section 2.1 (pi at
every multiple of L = floor(log2 y) plus the table of primes, stepping
through the primes from the sample), on the GPU, with the queries of the easy
leaves of pi(10^18) at alpha = 24: u = floor(X_b / m) for the single primes m
of a seeded sample of b.  Both lookups must agree with each other and with a
host count everywhere; their kernel times go to the test's output
(tests/device/pi_table_bench.hip)."""
import ctypes as C
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "device", "libpitable.so")
X, Y = 10**18, 24_000_000
NQ = 1 << 25


def tables():
    n = Y + 4096  # the primes table ends with a prime above every query
    is_p = np.ones(n + 1, dtype=bool)
    is_p[:2] = False
    for p in range(2, math.isqrt(n) + 1):
        if is_p[p]:
            is_p[p * p::p] = False
    primes = np.concatenate([[0], np.nonzero(is_p)[0]]).astype(np.uint32)  # 1-based
    pi_all = np.cumsum(is_p).astype(np.uint32)
    # bitmap: entry e covers the odd numbers 64e + 2j + 1, j < 32
    odd = is_p[1::2]
    odd = np.concatenate([odd, np.zeros((-len(odd)) % 32, dtype=bool)]).reshape(-1, 32)
    bits = np.packbits(odd, axis=1, bitorder="little").view("<u4").ravel()
    cnt = odd.sum(axis=1).astype(np.uint32)
    pre = np.concatenate([[0], np.cumsum(cnt)[:-1]]).astype(np.uint32)
    tab = np.stack([bits, pre], axis=1).astype(np.uint32).copy()
    L = int(math.floor(math.log2(Y)))
    samp = pi_all[np.arange(0, Y // L + 2) * L].astype(np.uint32)
    return primes, pi_all, tab, samp, L


def queries(primes, pi_all):
    """u = X_b // m over the single easy primes m of a seeded sample of b."""
    a = int(pi_all[Y])
    sq = math.isqrt(Y)
    b_lo = int(pi_all[sq]) + 1
    rng = np.random.default_rng(1503)
    out, total = [], 0
    for b in sorted(rng.choice(np.arange(b_lo, a), size=4096, replace=False)):
        p = int(primes[b])
        Xb = X // p
        tp = Xb // p
        m1 = max(Y // p + 1, p + 1)
        H = max(tp // p, Xb // (Y + 1))
        e1, e2 = max(H + 1, m1), min(tp, Y)
        if e1 > e2:
            continue
        s = math.isqrt(Xb)
        s = min(max(s + s // 2, e1 - 1), e2)
        k1, k2 = int(pi_all[e1 - 1]) + 1, int(pi_all[s])
        if k2 < k1:
            continue
        u = (Xb // primes[k1:k2 + 1].astype(np.uint64)).astype(np.uint32)
        out.append(u)
        total += len(u)
        if total >= NQ:
            break
    return np.concatenate(out)[:NQ].copy()


def test_bitmap_vs_sampled_pi_table():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is missing: run __graft_entry__.build()")
    primes, pi_all, tab, samp, L = tables()
    u = queries(primes, pi_all)
    assert int(u.min()) >= 2 and int(u.max()) <= Y
    import paper_1503_01839_amd as pc
    pc.lib()  # the HIP runtime the library uses is loaded first
    lib = C.CDLL(LIB)
    lib.pc_pi_table_bench.restype = C.c_int
    P = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    o1 = np.zeros(len(u), dtype=np.uint32)
    o2 = np.zeros(len(u), dtype=np.uint32)
    ms1, ms2 = C.c_float(), C.c_float()
    m = (1 << 32) // L + 1  # ceil(2^32 / L), L not a power of two
    print(f"case: pi lookups, {len(u)} queries, L = {L}", flush=True)
    rc = lib.pc_pi_table_bench(P(tab), C.c_uint64(len(tab)), P(samp), C.c_uint64(len(samp)),
                               C.c_uint32(m), P(primes), C.c_uint64(len(primes)), P(u),
                               C.c_uint64(len(u)), C.c_uint32(20), P(o1), P(o2),
                               C.byref(ms1), C.byref(ms2))
    assert rc == 0
    want = pi_all[u]
    assert np.array_equal(o1, want)
    assert np.array_equal(o2, want)
    steps = float(np.mean(want - samp[u // L]))
    bytes_tab, bytes_samp = tab.nbytes, samp.nbytes + primes.nbytes
    print(f"bitmap: {ms1.value:.3f} ms ({len(u) / ms1.value / 1e6:.2f} G lookups/s), "
          f"{bytes_tab / 2**20:.1f} MiB; sampled (L = {L}): {ms2.value:.3f} ms "
          f"({len(u) / ms2.value / 1e6:.2f} G lookups/s), {samp.nbytes / 2**20:.1f} MiB of samples "
          f"+ {primes.nbytes / 2**20:.1f} MiB of primes, {steps:.2f} prime steps per lookup",
          flush=True)

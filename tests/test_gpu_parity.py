"""GPU parity: the HIP path through the C ABI against the CPU oracle and the
paper's tables.  Every result is an integer, so every comparison is exact.
"""
import json
import os
import random
import sys

import pytest

import oracle as O

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_decomp.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)["records"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_small_x_table(pc):
    # x < 2^20 is answered from the device pi table
    say("case: small x table")
    rng = random.Random(3)
    xs = list(range(0, 300)) + [rng.randrange(0, 1 << 20) for _ in range(200)] + [(1 << 20) - 1]
    for x in xs:
        assert pc.pi_count(x) == O.pi_brute(x), x


def test_decompose_small_vs_oracle(pc):
    # tiny x through the sieve path, every component against the oracle
    rng = random.Random(5)
    cases = [(8, 2), (27, 3), (100, 4), (100, 10), (1000, 10), (1000, 31), (10**4, 21),
             (10**4, 100), (10**6, 100), (10**6, 200), (10**6, 1000), (30030, 31)]
    for _ in range(30):
        x = rng.randrange(64, 10**7)
        lo, hi = O.icbrt(x), O.isqrt(x)
        cases.append((x, rng.randrange(lo, hi + 1)))
    for x, y in cases:
        say("case: decompose", x, y)
        r = pc.decompose(x, y)
        o = O.decompose(x, y, 6, hard=O.HARD_SIEVE)
        assert (r.a, r.c, r.bmax) == (o.a, o.c, o.bmax), (x, y)
        assert r.s1 == o.s1, (x, y, "S1")
        assert r.s2_trivial == o.s2t, (x, y, "S2t")
        assert r.s2_easy == o.s2e, (x, y, "S2e")
        assert r.s2_hard == o.s2h, (x, y, "S2h")
        assert r.p2 == o.p2, (x, y, "P2")
        assert r.pi == O.pi_brute(x), (x, y)


def check_record(r, rec, what=""):
    assert (r.a, r.bmax) == (rec["a"], rec["bmax"]), (rec["x"], rec["y"], what)
    for got, key in ((r.s1, "s1"), (r.s2_trivial, "s2t"), (r.s2_easy, "s2e"),
                     (r.s2_hard, "s2h"), (r.p2, "p2"), (r.pi, "pi")):
        assert got == rec[key], (rec["x"], rec["y"], key, what)
    assert (r.n_trivial, r.n_easy, r.n_s1) == (rec["n_trivial"], rec["n_easy"], rec["n_s1"])
    if rec["n_hard"] is not None:
        assert r.n_hard == rec["n_hard"], (rec["x"], rec["y"], "n_hard", what)


def test_golden_records(pc):
    # every record, 1e8 to 1e18: the sieve route up to 1e13, Meissel's identity
    # with Table 1 above (Section 5)
    for rec in golden():
        say("case: golden", rec["x"], rec["y"], rec["route"])
        check_record(pc.decompose(rec["x"], rec["y"]), rec)


@pytest.mark.parametrize("seg,wg", [(32, 256), (32, 512), (64, 512), (64, 1024)])
def test_1e16_alpha_shape_grid(pc, seg, wg):
    # x = 1e16 with alpha in {1, 2, 4, 8} on every sieve shape, each component
    # against the oracle's record (S2h pinned to Table 1 by Meissel's identity)
    recs = {r["alpha"]: r for r in golden() if r["x"] == 10**16}
    for alpha in (1, 2, 4, 8):
        rec = recs[alpha]
        say("case: 1e16 grid", alpha, seg, wg)
        check_record(pc.decompose(10**16, rec["y"], segment_kib=seg, wg_size=wg), rec,
                     (alpha, seg, wg))


@pytest.mark.parametrize("seg,wg", [(32, 256), (32, 512), (64, 512), (64, 1024)])
def test_config_invariance(pc, seg, wg):
    # the sieve geometry never changes a value (the paper's own check, Section 5)
    for x, y in [(10**11, 4641), (10**12, 20000), (10**10 + 12345, 4000)]:
        say("case: invariance", x, y, seg, wg)
        o = O.decompose(x, y, 6, hard=O.HARD_SIEVE)
        for kw in (dict(flags=0), dict(flags=pc.FLAG_NO_BATCH_LARGE), dict(flags=pc.FLAG_TWO_PASS),
                   dict(small_span=64), dict(flags=pc.FLAG_TWO_PASS, small_span=64),
                   dict(tile_leaves=0xFFFFFFFF), dict(tile_leaves=2048)):
            r = pc.decompose(x, y, segment_kib=seg, wg_size=wg, **kw)
            assert (r.s2_hard, r.p2, r.pi) == (o.s2h, o.p2, o.pi), (x, y, seg, wg, kw)


def test_windows(pc):
    # a tiny carry budget forces many windows; carries must chain across them
    # (the stored counts of 1e12 at y = 1e4 take about 64 KiB in all)
    x, y = 10**12, 10**4
    o = O.decompose(x, y, 6, hard=O.HARD_SIEVE)
    for budget in (1 << 12, 1 << 14, 1 << 15):
        say("case: windows", budget)
        r = pc.decompose(x, y, carry_budget=budget)
        assert r.windows > 1
        assert (r.s2_hard, r.p2) == (o.s2h, o.p2), budget


def test_paper_powers_of_ten(pc, paper_pow10):
    # Table 1 up to 10^19, the largest power of ten below 2^64
    for n in range(1, 20):
        say("case: pi(10^%d)" % n)
        assert pc.pi_count(10**n) == paper_pow10[n], n


def test_paper_powers_of_two(pc, paper_pow2):
    # Table 2 up to 2^63, the largest power of two below 2^64
    for m in range(1, 64):
        say("case: pi(2^%d)" % m)
        assert pc.pi_count(2**m) == paper_pow2[m], m


def test_alpha_invariance(pc, paper_pow10):
    for n in (12, 13, 14):
        for alpha in (1, 2, 4, 8, 16):
            say("case: alpha", n, alpha)
            assert pc.pi_count(10**n, alpha) == paper_pow10[n], (n, alpha)


def test_random_vs_oracle(pc):
    rng = random.Random(1839)
    for _ in range(40):
        x = rng.randrange(1 << 20, 2 * 10**9)
        say("case: random", x)
        assert pc.pi_count(x) == O.pi_meissel(x), x


def test_bad_shapes_rejected(pc):
    with pytest.raises(pc.PicountError):
        pc.decompose(10**11, 4641, segment_kib=32, wg_size=1024)
    with pytest.raises(pc.PicountError):
        pc.decompose(10**11, 4641, segment_kib=128)


def test_p2_and_s2_hard_entry_points(pc):
    x, y = 10**11, 4641
    o = O.decompose(x, y, 6, hard=O.HARD_SIEVE)
    assert pc.s2_hard(x, y, o.a) == o.s2h
    assert pc.p2(x, y) == o.p2
    with pytest.raises(pc.PicountError):
        pc.s2_hard(x, y, o.a + 1)
    with pytest.raises(pc.PicountError):
        pc.p2(x, 10)  # y below icbrt(x)


@pytest.mark.parametrize("tile_leaves", [512, 4096, 49152, 0xFFFFFFFF])
def test_tile_split_invariance(pc, tile_leaves, paper_pow10):
    # cutting hot segments into column-range tiles never changes a value
    recs = {(r["x"], r["y"]): r for r in golden()}
    for (x, y) in [(10**12, 10**4), (10**13, 21544), (10**12, 80000)]:
        say("case: split", x, y, tile_leaves)
        rec = recs[(x, y)]
        for span in (0, 64):
            r = pc.decompose(x, y, tile_leaves=tile_leaves, small_span=span)
            assert (r.s2_hard, r.p2, r.pi) == (rec["s2h"], rec["p2"], rec["pi"]), \
                (x, y, tile_leaves, span)
            assert r.n_hard == rec["n_hard"]
            if tile_leaves == 512 and not span:
                assert r.tiles > r.segments
    say("case: split 1e15", tile_leaves)
    assert pc.pi_count_ex(10**15, tile_leaves=tile_leaves).pi == paper_pow10[15]


@pytest.mark.parametrize("small_kib", [4, 8])
@pytest.mark.parametrize("span", [1, 3, 64, 100000])
def test_small_segment_invariance(pc, small_kib, span):
    # the boundary between one-wavefront and workgroup segments moves nothing
    recs = {(r["x"], r["y"]): r for r in golden()}
    for (x, y) in [(10**12, 20000), (10**11, 4641), (10**13, 21544)]:
        say("case: small segments", x, y, small_kib, span)
        rec = recs[(x, y)]
        r = pc.decompose(x, y, small_kib=small_kib, small_span=span)
        assert (r.s2_hard, r.p2, r.pi) == (rec["s2h"], rec["p2"], rec["pi"]), (x, y)
        assert r.n_hard == rec["n_hard"]
        assert r.small_segments > 0

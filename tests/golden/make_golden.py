"""Write tests/golden/oracle_decomp.json: the oracle's decomposition of pi(x)
at the configurations the GPU parity tests use.

Calls nothing but the CPU oracle (``oracle/``) and the paper's Table 1.

* route "sieve"    : every term from the oracle; S2h by its direct segmented
                     sieve (x <= 1e13, minutes at most).
* route "identity" : S1, S2t, S2e and P2 from the oracle; S2h from Meissel's
                     identity with the paper's tabulated pi(x) (Table 1):
                     S2h = pi(x) - a + 1 + P2 - S1 - S2t - S2e.
                     --tuned records take S1 and P2 from oracle.s1_p2 and
                     S2t, S2e as sums of oracle.leaf_sample over slices of b
                     run in parallel (the same leaf routine as the whole
                     decomposition; n_hard is then not counted).
Usage: python tests/golden/make_golden.py [--big] [--tuned]
  --big   adds 1e16 (alpha 1, 2, 4, 8) and 1e18 (alpha 8, 16)
  --tuned adds the alphas the library picks by default: 1e16 (16), 1e17 (24),
          1e18 (36; and 24 and 28, the defaults of earlier kernels)
  --only-tuned  skips the small sieve-route records (they are kept from the
          existing file)
  --only-missing  skips every record whose (x, y) the existing file already holds
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402

C = 6


def paper_pow10():
    out = {}
    with open(os.path.join(HERE, "paper_pi_pow10.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, v = line.split()
                out[int(n)] = int(v)
    return out


def job(spec):
    x, alpha, route, n10 = spec
    r = O.icbrt(x)
    y = min(alpha * r, O.isqrt(x))
    if route == "sieve":
        d = O.decompose(x, y, C, hard=O.HARD_SIEVE)
        s2h = d.s2h
    else:
        d = O.decompose(x, y, C, hard=O.HARD_NONE)
        pi = paper_pow10()[n10]
        s2h = pi - d.a + 1 + d.p2 - d.s1 - d.s2t - d.s2e
    rec = dict(x=x, alpha=alpha, y=y, c=d.c, a=d.a, z=d.z, bmax=d.bmax, s1=d.s1, s2t=d.s2t,
               s2e=d.s2e, s2h=s2h, p2=d.p2, n_s1=d.n_s1, n_trivial=d.n_trivial,
               n_easy=d.n_easy, n_hard=d.n_hard, n_p2=d.n_p2, route=route)
    rec["pi"] = d.s1 + d.s2t + d.s2e + s2h + d.a - 1 - d.p2
    if route == "identity":
        rec["source"] = f"S2h from Meissel's identity with pi(10^{n10}) of Table 1"
    print(json.dumps(rec), flush=True)
    return rec


def _slice(args):
    x, y, b0, b1 = args
    d = O.leaf_sample(x, y, C, b0, b1, 0)
    return d.s2t, d.s2e, d.n_trivial, d.n_easy


def job_sliced(x, alpha, n10, ex, nslices=96):
    """An identity record with the special leaves summed slice by slice."""
    r = O.icbrt(x)
    y = min(alpha * r, O.isqrt(x))
    base = O.s1_p2(x, y, C)
    a = base.a
    cuts = [C + 1 + (a - C - 1) * k // nslices for k in range(nslices + 1)]
    # small b have the most candidates m: cut them finer
    cuts = sorted(set([C + 1 + k for k in range(0, 64, 4)] + cuts))
    parts = list(ex.map(_slice, [(x, y, b0, b1) for b0, b1 in zip(cuts, cuts[1:]) if b0 < b1]))
    s2t = sum(p[0] for p in parts)
    s2e = sum(p[1] for p in parts)
    pi = paper_pow10()[n10]
    s2h = pi - a + 1 + base.p2 - base.s1 - s2t - s2e
    rec = dict(x=x, alpha=alpha, y=y, c=base.c, a=a, z=base.z, bmax=base.bmax, s1=base.s1,
               s2t=s2t, s2e=s2e, s2h=s2h, p2=base.p2, n_s1=base.n_s1,
               n_trivial=sum(p[2] for p in parts), n_easy=sum(p[3] for p in parts),
               n_hard=None, n_p2=base.n_p2, route="identity")
    rec["pi"] = base.s1 + s2t + s2e + s2h + a - 1 - base.p2
    rec["source"] = f"S2h from Meissel's identity with pi(10^{n10}) of Table 1"
    print(json.dumps(rec), flush=True)
    return rec


TUNED = ((10**16, 16, 16), (10**17, 24, 17), (10**18, 24, 18), (10**18, 28, 18), (10**18, 36, 18))


def y_of(x, alpha):
    return min(alpha * O.icbrt(x), O.isqrt(x))


def main():
    path = os.path.join(HERE, "oracle_decomp.json")
    old = []
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)["records"]
    have = {(r["x"], r["y"]) for r in old} if "--only-missing" in sys.argv else set()
    specs = []
    if "--only-tuned" not in sys.argv:
        for n in (8, 9, 10, 11, 12):
            for alpha in (1, 2, 4, 8):
                specs.append((10**n, alpha, "sieve", n))
        specs.append((10**13, 1, "sieve", 13))
        specs.append((2**40, 3, "sieve", None))
    if "--big" in sys.argv:
        for alpha in (1, 2, 4, 8):
            specs.append((10**16, alpha, "identity", 16))
        specs.append((10**18, 8, "identity", 18))
        specs.append((10**18, 16, "identity", 18))
    specs = [s for s in specs if (s[0], y_of(s[0], s[1])) not in have]
    # largest first so the pool finishes together
    specs.sort(key=lambda s: -s[0] / s[1])
    with ProcessPoolExecutor(max_workers=int(os.environ.get("GOLDEN_JOBS", "6"))) as ex:
        recs = list(ex.map(job, specs))
        if "--tuned" in sys.argv:
            for x, alpha, n10 in TUNED:
                if (x, y_of(x, alpha)) not in have:
                    recs.append(job_sliced(x, alpha, n10, ex))
    recs.sort(key=lambda r: (r["x"], r["alpha"]))
    pw = paper_pow10()
    for r in recs:  # every record must reproduce the paper where the paper has a value
        for n, v in pw.items():
            if r["x"] == 10**n:
                assert r["pi"] == v, r
    keep = {(r["x"], r["y"]): r for r in old}
    for r in recs:
        keep[(r["x"], r["y"])] = r
    out = sorted(keep.values(), key=lambda r: (r["x"], r["y"]))
    with open(path, "w") as f:
        json.dump({"comment": "written by tests/golden/make_golden.py from oracle/ only; "
                              "c = 6 (wheel 2*3*5*7*11*13); y = min(alpha*icbrt(x), isqrt(x))",
                   "records": out}, f, indent=1)
    print("wrote", path, len(out))


if __name__ == "__main__":
    main()

"""Write tests/golden/oracle_pi_mixes.json: pi(x) by the CPU oracle for the
members of the seeded many-query workloads that the oracle finishes in
seconds, so that batch and serving results are checked against an
independent computation, not only against the GPU's own per-query path.

Calls nothing but the CPU oracle (``oracle/``) and the seeded input
generators (``paper_1503_01839_amd.workloads``, inputs only).

* batch_4096: the batch workload (4096 x log-uniform in [1e8, 1e15], seed
  1503): every x <= 1e13, and 64 members above 1e13 drawn with seed 1839.
* serve_test: the request stream of the GPU serving test (160 x log-uniform
  in [1e8, 1e13], seed 1839): every x.

Each value is oracle.decompose(x, y, 6, HARD_SIEVE).pi with y = 16 icbrt(x)
(clamped to isqrt x); pi(x) does not depend on y.

Usage: python tests/golden/make_mix_golden.py   (GOLDEN_JOBS processes, default 8)
"""
import json
import os
import random
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1503_01839_amd import workloads as W  # noqa: E402


def pi_of(x):
    if x < 8:
        return x, O.pi_brute(x)
    y = min(16 * O.icbrt(x), O.isqrt(x))
    return x, O.decompose(x, y, 6, hard=O.HARD_SIEVE).pi


def main():
    batch = W.batch_queries(4096)
    small = sorted({x for x in batch if x <= 10**13})
    big = sorted({x for x in batch if x > 10**13})
    big = sorted(random.Random(1839).sample(big, 64))
    serve_xs, _ = W.serve_stream(160, rate_per_s=400.0, lo_exp=8.0, hi_exp=13.0, seed=1839)
    todo = sorted(set(small) | set(big) | set(serve_xs), reverse=True)
    with ProcessPoolExecutor(max_workers=int(os.environ.get("GOLDEN_JOBS", "8"))) as ex:
        vals = dict(ex.map(pi_of, todo))
    out = {"comment": "pi(x) by oracle.decompose (HARD_SIEVE, y = 16 icbrt x); written by "
                      "tests/golden/make_mix_golden.py from oracle/ only",
           "batch_4096": [[x, vals[x]] for x in small + big],
           "serve_test": [[x, vals[x]] for x in sorted(set(serve_xs))]}
    path = os.path.join(HERE, "oracle_pi_mixes.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path, len(out["batch_4096"]), len(out["serve_test"]))


if __name__ == "__main__":
    main()

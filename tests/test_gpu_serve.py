"""Serving on the GPU: every answer of a replayed request stream is the same
as the request run alone, whether requests are batched as they arrive, served
one at a time (the plain per-query server), or sent to the windowed path;
latencies are non-negative.  Inputs: x log-uniform and Poisson arrivals from
fixed seeds."""
import json
import os

import pytest

from paper_1503_01839_amd import workloads as W

MIXES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_pi_mixes.json")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def stream(n, rate, lo, hi, seed):
    return W.serve_stream(n, rate_per_s=rate, lo_exp=lo, hi_exp=hi, seed=seed)


def test_serve_equals_solo(pc):
    xs, t = stream(160, 400.0, 8.0, 13.0, 1839)
    say("case: serve", len(xs))
    solo = [pc.pi_count(x) for x in xs]
    pis, lat, st = pc.serve(xs, t)
    assert pis == solo
    assert min(lat) >= 0 and st["rounds"] >= 1
    pis1, lat1, st1 = pc.serve(xs, t, max_inflight=1, max_round=1)
    assert pis1 == solo and st1["rounds"] == sum(1 for x in xs if x >= 2**20)
    pis2, _, _ = pc.serve(xs, t, flags=pc.FLAG_NO_GRAPH, max_inflight=2, max_round=16)
    assert pis2 == solo
    # and every answer equals the oracle's pi(x)
    with open(MIXES) as f:
        want = dict(map(tuple, json.load(f)["serve_test"]))
    assert [want[x] for x in xs] == pis


def test_serve_windowed_requests(pc):
    # a one-byte memory budget: no request's counts fit a round, so every
    # request (x >= 2^20) goes through the windowed path
    xs, t = stream(24, 200.0, 9.0, 12.0, 5)
    say("case: serve windowed")
    solo = [pc.pi_count(x) for x in xs]
    pis, lat, st = pc.serve(xs, t, mem_budget=1)
    assert pis == solo
    assert st["windowed"] == sum(1 for x in xs if x >= 2**20)


def test_serve_rejects_bad_arrivals(pc):
    with pytest.raises(pc.PicountError):
        pc.serve([10**9, 10**9], [1.0, 0.5])
    with pytest.raises(pc.PicountError):
        pc.serve([10**9], [float("nan")])

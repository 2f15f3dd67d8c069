#!/usr/bin/env python3
"""Benchmark: pi(1e18) on one MI355X through the C ABI.

A step is one complete pi(x) evaluation at x = 1e18: device tables (primes and
pi up to sqrt x, mu*lpf up to y, wheel), S1, trivial and easy leaves, the
segmented sieve with hard leaves and P2, the carry scan and the final
combination.  The input is the single integer x, resident before timing.

--x runs the same step at another size (the other single-query
configurations, e.g. x = 2^63 + 2^61); the default is the headline, 1e18.

Every step (warm-up steps included) is checked: pi(x) against the paper's
Table 1 / Table 2 where they hold x, and pi with S1, S2t, S2e, S2h and P2
against the oracle's record for the same (x, y) in tests/golden where there is
one; every step must also agree with the first.  Each step's values go to
stderr.  On any disagreement the JSON line carries "value": null and the
mismatches, and the exit status is 3.

Prints one JSON line.  `value` is special leaves (trivial + easy + hard, the
whole S2 tree at the chosen alpha) per second of pi(1e18) wall time; the
alpha-independent pi(x) wall time is `ms_per_step`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "S2 special leaves/s + π(x) wall time at x=1e18; batched queries/s, p50/p99"
X = 10**18
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")

# MI355X: 256 CUs of 64 lanes at 2.4 GHz: one 32-bit integer operation per lane
# per clock (the sieve is integer work; no matrix cores, no packed math).
CUS, LANES, CLOCK_HZ = 256, 64, 2.4e9
INT_PEAK = CUS * LANES * CLOCK_HZ  # 32-bit integer lane operations per second

# Algorithmic integer operations of the sieve kernel, per unit of work:
#   crossing an odd multiple of p_b: address, mask, one LDS read-modify-write
#   placing prime p_b in a segment: first multiple by multiply-high reciprocal
#   a hard leaf or a P2 lookup: 64/32 division by reciprocal (about 12), a
#   prefix-table read with a masked popcount (4), the signed add (2)
OPS_CROSSING, OPS_VISIT, OPS_LEAF = 3, 8, 18
# ... and of the easy-leaf kernel, per work item (one easy leaf, or a run of
# them sharing pi(u)): a quotient by the fp64 reciprocal with its remainder
# correction (about 12), a pi-table lookup (4), the signed add (2)
OPS_EASY_ITEM = 18

# Bounded oracle sample of the same workload (same x and y as the GPU line):
# the special leaves of every B_STEP-th prime p_b (b = 7, 7 + B_STEP, ...)
# of all three classes, the hard ones only with u <= U_MAX.
B_STEP, U_MAX = 64, 10**8

# Whole queries the oracle finishes in seconds, timed beside the GPU at the
# same x and y (the y the library picks for that x).
WHOLE_QUERY_X = (10**11, 10**12)

# Batch and serving workloads (paper_1503_01839_amd.workloads): 4096 queries
# log-uniform in [1e8, 1e15] (seed 1503); a Poisson stream log-uniform in
# [1e10, 1e18] (seed 1839) at a rate frozen at 0.8 x the batched throughput
# measured on that mix (25.4 queries/s for 1000 requests on MI355X).
BATCH_N = 4096
SERVE_RATE = 20.3
SERVE_TOTAL = 20000  # the stream's full length; the default run serves a prefix

# HBM traffic of the sieve kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
# scaled by the same counters on a plain copy of known size; reported only while
# the kernel source is the one the counters were taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sieve_traffic_1e18.txt")
PEAKS_FILE = os.path.join(ROOT, "profiles", "gpu_peaks_microbench.txt")
KERNEL_SRC = [os.path.join(ROOT, "paper_1503_01839_amd", "csrc", f)
              for f in ("pc_sieve.hip", "pc_leafrange.h", "pc_block.h", "pc_device.h",
                        "pc_internal.h")]


def kernel_sha256():
    """Hash of the sources the sieve kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def icbrt(n: int) -> int:
    """floor(n^(1/3))."""
    r = int(round(n ** (1.0 / 3.0)))
    while r ** 3 > n:
        r -= 1
    while (r + 1) ** 3 <= n:
        r += 1
    return max(r, 1)


def read_pairs(name):
    out = {}
    with open(os.path.join(GOLDEN_DIR, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[int(k)] = int(v)
    return out


def expected_pi(x):
    """pi(x) from the paper's Table 1 (10^n) or Table 2 (2^m), else None."""
    for name, base in (("paper_pi_pow10.txt", 10), ("paper_pi_pow2.txt", 2)):
        for k, v in read_pairs(name).items():
            if base ** k == x:
                return v
    return None


def golden_record(x, y):
    """The oracle's decomposition of (x, y) from tests/golden, or None."""
    with open(os.path.join(GOLDEN_DIR, "oracle_decomp.json")) as f:
        for rec in json.load(f)["records"]:
            if rec["x"] == x and rec["y"] == y:
                return rec
    return None


def parts(r):
    return {"pi": r.pi, "s1": r.s1, "s2t": r.s2_trivial, "s2e": r.s2_easy, "s2h": r.s2_hard,
            "p2": r.p2}


def check_step(tag, r, pi_want, rec, first):
    """Mismatches of one step against the table, the golden record and the
    first step."""
    bad = []
    got = parts(r)
    if pi_want is not None and r.pi != pi_want:
        bad.append({"step": tag, "what": "pi vs paper table", "got": r.pi, "want": pi_want})
    if rec is not None:
        for k in ("pi", "s1", "s2t", "s2e", "s2h", "p2"):
            if got[k] != rec[k]:
                bad.append({"step": tag, "what": f"{k} vs oracle record", "got": got[k],
                            "want": rec[k]})
    if first is not None and got != first:
        bad.append({"step": tag, "what": "differs from the first step", "got": got,
                    "want": first})
    return bad


def lds_rmw_peak():
    """LDS atomic read-modify-writes per second of this GPU in the crossing
    pattern, from the committed micro-benchmark summary, or None."""
    try:
        kv = dict(line.split(":", 1) for line in open(PEAKS_FILE) if ":" in line)
        return float(kv["lds_atomic_crossing_per_s"])
    except (OSError, KeyError, ValueError):
        return None


def traffic_bytes(x, y):
    """HBM bytes per sieve launch from the committed counter summary, or None
    when there is none, it was taken on another (x, y), or the kernel source
    has changed since."""
    try:
        kv = dict(line.split(":", 1) for line in open(TRAFFIC_FILE) if ":" in line)
    except OSError:
        return None
    if kv.get("kernel_sha256", "").strip() != kernel_sha256():
        return None
    if kv.get("workload_x_y", "").split() != [str(x), str(y)]:
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(nbytes):
    """One plain device-to-device copy of nbytes through the HIP runtime the
    library links (for scaling HBM counters)."""
    import ctypes as C
    import paper_1503_01839_amd as pc
    pc.lib()
    L = C.CDLL("libamdhip64.so.7")
    L.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    L.hipMemset.argtypes = [C.c_void_p, C.c_int, C.c_size_t]
    L.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    L.hipFree.argtypes = [C.c_void_p]
    a, b = C.c_void_p(), C.c_void_p()
    for p in (a, b):
        if L.hipMalloc(C.byref(p), nbytes) != 0:
            raise SystemExit("hipMalloc failed")
    L.hipMemset(a, 1, nbytes)
    L.hipDeviceSynchronize()
    if L.hipMemcpy(b, a, nbytes, 3) != 0:  # device to device
        raise SystemExit("hipMemcpy failed")
    L.hipDeviceSynchronize()
    L.hipFree(a)
    L.hipFree(b)
    print(json.dumps({"copy_bytes": nbytes}), flush=True)


def batch_leg(pc, n):
    """n queries in batch rounds (one HIP graph per round) against the plain
    per-query path, same inputs; results must agree."""
    from paper_1503_01839_amd import workloads as W
    xs = W.batch_queries(n)
    pc.pi_count_batch(xs[:64])
    t0 = time.perf_counter()
    rb = pc.pi_count_batch(xs)
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    rs = pc.pi_count_batch(xs, flags=pc.FLAG_BATCH_SEQUENTIAL)
    ts = time.perf_counter() - t0
    if rb != rs:
        raise SystemExit("batch results differ from the per-query path")
    return {"queries": n, "x": "log-uniform [1e8, 1e15], PCG64(1503)", "queries_per_s": n / tb,
            "ms": tb * 1e3, "plain_queries_per_s": n / ts, "plain_ms": ts * 1e3,
            "speedup": ts / tb, "match_plain": True}


def serve_leg(pc, n, modes=("served", "plain"), piece=0):
    """An open-loop Poisson stream served with continuous batching, and by the
    one-request-at-a-time server; p50/p99 of completion - arrival.  piece > 0
    replays the stream in consecutive pieces of that many requests (each
    piece's arrival times re-based to its first), one call each, so that a
    long stream reports progress; the latencies of all pieces are pooled."""
    import hashlib
    import numpy as np
    from paper_1503_01839_amd import workloads as W
    xs, arr = W.serve_stream(n, rate_per_s=SERVE_RATE)
    pc.pi_count_batch(xs[:16])
    out = {"requests": n,
           "stream": (f"the first {n} of the {SERVE_TOTAL}-request stream" if n < SERVE_TOTAL
                      else f"the whole {SERVE_TOTAL}-request stream"),
           "x": "log-uniform [1e10, 1e18], PCG64(1839)",
           "arrivals": f"Poisson, {SERVE_RATE}/s"}
    if piece:
        out["piece_requests"] = piece
    kwargs = {"served": {}, "plain": dict(max_inflight=1, max_round=1)}
    ref = None
    for name in modes:
        step = piece or n
        pis, lat, wall = [], [], 0.0
        agg = dict(rounds=0, windowed=0, max_round_size=0, max_inflight_seen=0)
        for k in range(0, n, step):
            t0 = arr[k]
            p_pis, p_lat, st = pc.serve(xs[k:k + step], [t - t0 for t in arr[k:k + step]],
                                        **kwargs[name])
            pis += p_pis
            lat += p_lat
            wall += st["wall_s"]
            for f in ("rounds", "windowed"):
                agg[f] += st[f]
            for f in ("max_round_size", "max_inflight_seen"):
                agg[f] = max(agg[f], st[f])
            if piece:
                print(f"serve {name}: {min(k + step, n)}/{n} requests", file=sys.stderr, flush=True)
        if ref is None:
            ref = pis
        elif pis != ref:
            raise SystemExit("served results differ from the per-request server")
        lat = np.array(lat) * 1e3
        out[name] = {"requests_per_s": n / wall, "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "rounds": agg["rounds"],
                     "windowed": agg["windowed"], "max_round": agg["max_round_size"],
                     "max_inflight": agg["max_inflight_seen"],
                     "results_sha256": hashlib.sha256(np.array(pis, dtype=np.uint64).tobytes())
                     .hexdigest()}
    return out


def _sample_part(args):
    x, y, b0, step, umax = args
    import oracle
    t0 = time.perf_counter()
    d = oracle.leaf_sample(x, y, 6, b0, 1 << 62, umax, b_step=step)
    return d.n_trivial, d.n_easy, d.n_hard, d.s2t, d.s2e, d.s2h, time.perf_counter() - t0


def cpu_threads():
    """Host threads this process may use (the box's share, at most 16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_pool():
    """Worker processes for the oracle sample, forked before this process
    touches the GPU (the children never use it)."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    n = cpu_threads()
    ex = ProcessPoolExecutor(max_workers=n, mp_context=multiprocessing.get_context("fork"))
    list(ex.map(abs, range(n)))  # start every worker now
    return ex, n


def cpu_baseline(pool, x, y):
    """The oracle on a bounded sample of the same query: the special leaves of
    every B_STEP-th prime, all classes (hard ones with u <= U_MAX), once on
    one thread and once split over every host thread (one process each)."""
    ex, n = pool
    one = ex.submit(_sample_part, (x, y, 7, B_STEP, U_MAX)).result()
    leaves = one[0] + one[1] + one[2]
    t0 = time.perf_counter()
    got = list(ex.map(_sample_part, [(x, y, 7 + i * B_STEP, n * B_STEP, U_MAX)
                                     for i in range(n)]))
    t_all = time.perf_counter() - t0
    ex.shutdown()
    if [sum(g[k] for g in got) for k in range(6)] != list(one[:6]):
        raise SystemExit("the split oracle sample differs from the single-thread sample")
    return {"value": leaves / t_all, "unit": "special leaves/s", "cores": n, "kind": "oracle",
            "nproc": os.cpu_count(), "single_thread_value": leaves / one[6],
            "single_thread_s": one[6], "all_threads_s": t_all,
            "sample": (f"pi({x:.0e}) at the GPU line's y = {y}: the special leaves of every "
                       f"{B_STEP}th prime p_b (b = 7, {7 + B_STEP}, ...), hard ones only with "
                       f"u <= {U_MAX:.0e}: {one[0]} trivial + {one[1]} easy + {one[2]} hard; "
                       f"C oracle, {n} processes (each its own tables) and one")}


def whole_query_oracle(pc):
    """Whole pi(x) decompositions the oracle finishes in seconds, beside the
    GPU's time at the same x and y."""
    import oracle
    out = []
    for x in WHOLE_QUERY_X:
        r = pc.pi_count_ex(x)
        g = min(pc.pi_count_ex(x).ms_total for _ in range(3))
        t0 = time.perf_counter()
        d = oracle.decompose(x, r.y, 6, hard=oracle.HARD_SIEVE)
        t = time.perf_counter() - t0
        if (d.s1, d.s2t, d.s2e, d.s2h, d.p2) != (r.s1, r.s2_trivial, r.s2_easy, r.s2_hard, r.p2):
            raise SystemExit(f"oracle and GPU differ at x = {x}")
        out.append({"x": x, "y": r.y, "pi": r.pi, "oracle_s": t, "oracle_threads": 1,
                    "gpu_ms": g, "ratio": t / (g / 1e3)})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--x", type=int, default=X,
                    help="the single query (default 1e18, the headline; other sizes for the "
                         "other single-query configurations, e.g. 2^63 + 2^61)")
    ap.add_argument("--alpha", type=float, default=0.0, help="0 = library's tuned value")
    ap.add_argument("--segment-kib", type=int, default=0)
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--keep-tables", action="store_true",
                    help="reuse device tables across steps (default: rebuild every step)")
    ap.add_argument("--carry-budget", type=int, default=0, metavar="BYTES",
                    help="bytes of stored counts per window of segments; 0 = library default")
    ap.add_argument("--seeded", action="store_true",
                    help="seed every window on its own with phi(m_min, b) (Section 4)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-queries", type=int, default=BATCH_N, help="0 = skip the batch leg")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help=f"requests of the serving leg (the full stream is {SERVE_TOTAL}); 0 = skip")
    ap.add_argument("--serve-modes", default="served,plain",
                    help="servers of the serving leg: served (continuous batching), plain")
    ap.add_argument("--serve-piece", type=int, default=0,
                    help="replay the stream in pieces of this many requests (0 = one call)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one plain device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(pi(x) shards by segment range, see DESIGN.md); rerun with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    modes = tuple(m for m in args.serve_modes.split(",") if m)
    if not modes or any(m not in ("served", "plain") for m in modes):
        raise SystemExit("--serve-modes takes served and/or plain")
    if args.serve_piece < 0 or not 0 <= args.x <= 2**72:
        raise SystemExit("--serve-piece must be >= 0 and --x in [0, 2^72]")
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    pool = None if args.no_cpu_baseline else oracle_pool()
    import paper_1503_01839_amd as pc

    flags = 0 if args.keep_tables else pc.FLAG_REBUILD_TABLES
    if args.seeded:
        flags |= pc.FLAG_SEEDED
    cfg = dict(alpha=args.alpha, segment_kib=args.segment_kib, wg_size=args.wg, flags=flags,
               carry_budget=args.carry_budget)
    default_knobs = not (args.seeded or args.carry_budget or args.alpha or args.segment_kib
                         or args.wg)
    x = args.x
    pi_want = expected_pi(x)
    rec = None
    bad = []
    first = None

    def step(tag):
        nonlocal rec, first
        r = pc.pi_count_wide(x, **cfg) if x >= 2**64 else pc.pi_count_ex(x, **cfg)
        if first is None:
            rec = golden_record(x, r.y)
        bad.extend(check_step(tag, r, pi_want, rec, first))
        if first is None:
            first = parts(r)
        print(f"{tag}: {r.ms_total:.1f} ms (tables {r.ms_tables:.1f}, leaves {r.ms_leaves:.1f}, "
              f"sieve {r.ms_sieve:.1f}) pi={r.pi} S1={r.s1} S2t={r.s2_trivial} "
              f"S2e={r.s2_easy} S2h={r.s2_hard} P2={r.p2}", file=sys.stderr, flush=True)
        return r

    for i in range(args.warmup):
        step(f"warmup {i}")
    results = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        results.append(step(f"step {i}"))
    wall = time.perf_counter() - t0  # every call returns with its result on the host
    r = results[-1]
    ms_step = 1e3 * wall / args.steps
    leaves = r.n_trivial + r.n_easy + r.n_hard

    # roofline of the dominant kernel (the sieve): algorithmic integer operations
    k_ms = sum(q.ms_k_sieve for q in results) / len(results)
    launches = r.sieve_launches
    avg_launch_ms = k_ms / max(launches, 1)
    visits = r.segments * (r.bmax - r.c)
    ops = (OPS_CROSSING * r.crossings + OPS_VISIT * visits + OPS_LEAF * (r.n_hard + r.n_p2))
    ops_per_launch = ops / max(launches, 1)
    achieved = ops_per_launch / (avg_launch_ms / 1e3)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": INT_PEAK / 1e12,
            "unit": "T int-ops/s", "frac": achieved / INT_PEAK,
            "traffic": traffic_bytes(x, r.y) if x == X and default_knobs else None,
            "kernel": "k_sieve", "launches": launches, "avg_launch_ms": avg_launch_ms,
            "ops_per_launch": ops_per_launch,
            "work": {"crossings": r.crossings, "prime_visits": visits, "hard_leaves": r.n_hard,
                     "p2_lookups": r.n_p2,
                     "ops_per_unit": {"crossing": OPS_CROSSING, "visit": OPS_VISIT,
                                      "leaf": OPS_LEAF}}}
    # the same kernel against its LDS bound: one atomic read-modify-write per
    # crossing, at the measured rate of the crossing pattern
    lds_peak = lds_rmw_peak()
    rmw = r.crossings / max(launches, 1)
    roof_lds = None if not lds_peak else {
        "bound": "lds", "achieved": rmw / (avg_launch_ms / 1e3) / 1e12, "peak": lds_peak / 1e12,
        "unit": "T LDS RMW/s", "frac": rmw / (avg_launch_ms / 1e3) / lds_peak, "kernel": "k_sieve",
        "peak_source": "profiles/gpu_peaks_microbench.txt", "rmw_per_launch": rmw}
    e_ms = sum(q.ms_k_easy for q in results) / len(results)
    e_ops = OPS_EASY_ITEM * r.n_easy_items
    roof_easy = {"bound": "alu", "achieved": e_ops / (e_ms / 1e3) / 1e12 if e_ms else None,
                 "peak": INT_PEAK / 1e12, "unit": "T int-ops/s",
                 "frac": e_ops / (e_ms / 1e3) / INT_PEAK if e_ms else None,
                 "kernel": "k_easy", "launches": 1, "avg_launch_ms": e_ms,
                 "work": {"items": r.n_easy_items, "easy_leaves": r.n_easy,
                          "ops_per_item": OPS_EASY_ITEM}}

    ok = not bad
    out = {
        "metric": METRIC, "value": leaves / (ms_step / 1e3) if ok else None,
        "unit": "special leaves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64/i128",
        "data": "synthetic",
        "config": {"workload": ("pi(x) single query, x = 1e18 (Table 1 row 10^18)" if x == X
                                else f"pi(x) single query, x = {x}"), "x": x,
                   "alpha": r.y / icbrt(x), "y": r.y, "a": r.a, "c": r.c, "z": r.z, "bmax": r.bmax,
                   "segment_bits": r.segment_bits, "segments": r.segments,
                   "windows": r.windows, "carry_budget": args.carry_budget or "default",
                   "windows_seeded": args.seeded,
                   "tables_rebuilt_each_step": not args.keep_tables},
        "pi": r.pi, "parts": parts(r),
        "checked_against": {"paper_table": pi_want is not None,
                            "oracle_record": rec is not None,
                            "steps": args.warmup + args.steps},
        "pi_matches_table": (all(q.pi == pi_want for q in results) if pi_want is not None
                             else None),
        "all_steps_equal": not any(b["what"] == "differs from the first step" for b in bad),
        "pi_wall_ms": ms_step,
        "leaves": {"trivial": r.n_trivial, "easy": r.n_easy, "hard": r.n_hard,
                   "easy_items": r.n_easy_items, "s1_terms": r.n_s1, "p2_terms": r.n_p2},
        "hard_leaves_per_s": r.n_hard / (ms_step / 1e3),
        "easy_hard_leaves_per_s": (r.n_easy + r.n_hard) / (ms_step / 1e3),
        "sieve_bits_per_s": (r.segments * r.segment_bits) / (ms_step / 1e3),
        "crossings_per_s": r.crossings / (ms_step / 1e3),
        "phase_ms": {"tables": r.ms_tables, "leaves": r.ms_leaves, "sieve": r.ms_sieve,
                     "k_sieve": r.ms_k_sieve, "k_scan": r.ms_k_scan, "k_easy": r.ms_k_easy,
                     "k_s1": r.ms_k_s1, "k_seed": r.ms_k_seed},
        "device_bytes": r.device_bytes,
        "roofline": roof,
        "roofline_easy": roof_easy,
        "roofline_lds": roof_lds,
        "paper_context": "Table 3: pi(1e18) took 108 node-s (v2015.01.30) on 2x Xeon E5-2670 "
                         "(16 cores); not a target",
    }
    if not ok:
        out["error"] = "a step's result disagrees with the paper, the oracle or the first step"
        out["mismatches"] = bad[:20]
        print(json.dumps(out), flush=True)
        if pool:
            pool[0].shutdown()
        sys.exit(3)
    if args.batch_queries:
        out["batch"] = batch_leg(pc, args.batch_queries)
    if args.serve_requests:
        out["serve"] = serve_leg(pc, args.serve_requests, modes, args.serve_piece)
    if not args.no_cpu_baseline and x >= 2**64:
        out["cpu_baseline"] = None
        out["cpu_baseline_note"] = "the oracle takes x < 2^64 only"
    elif not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pool, x, r.y)
        out["whole_query_oracle"] = whole_query_oracle(pc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

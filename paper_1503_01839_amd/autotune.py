"""Autotuner for alpha = y / icbrt(x), the knob that moves work between the
sieve (which shrinks as alpha grows: z = x / y) and the easy leaves (which
grow), and for the sieve's shape (LDS segment size and workgroup size).  For
each half decade of x it times pi(x) at every candidate alpha on this GPU
(tables cached, median of repeats, default shape), then every shape at the
best alpha, and writes the winners to csrc/pc_alpha_table.h, the table the
library reads when alpha = 0 (alpha) and when the caller names no shape.

A batch fills the GPU with many queries at once, so what counts there is the
total work rather than one query's latency: the batch alpha of a half decade
(up to 10^16; above, a query fills the GPU alone and takes the single-query
alpha) is the one that runs a batch of queries log-uniform in that half
decade (seeded) in the least time.

    python -m paper_1503_01839_amd.autotune              # tune, write the header
    python -m paper_1503_01839_amd.autotune --dry-run    # tune, print only
    python -m paper_1503_01839_amd.autotune --batch-only # batch alphas; keep the rest
    python -m paper_1503_01839_amd.autotune --sweep 16 --alphas 1,2,4,8
                                            # every alpha x shape at x = 10^16, print only

Every candidate's result is checked before its time counts: pi(x) must be the
same at every alpha and shape of a half decade (the paper's own check of its
values, Section 5), must equal Table 1 where x is a power of ten, and a
batch must return the same values at every alpha it is timed at; any
disagreement stops the tuner.  Segments of 128 KiB are not among the shapes:
the library builds 32 and 64 KiB segments only (the 64 KiB ones already run
35-60% slower than 32 KiB at 1e18 and 1e19, and 128 KiB would leave one
workgroup per CU).

Rebuild the library afterwards (__graft_entry__.build())."""
from __future__ import annotations

import argparse
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "csrc", "pc_alpha_table.h")
ALPHAS = [1, 1.5, 2, 3, 4, 6, 8, 12, 16, 24, 28, 32, 36, 40, 48, 64, 96]
SHAPES = [(32, 512), (32, 256), (64, 512), (64, 1024)]  # (segment KiB, workgroup threads)
BATCH_HI = 16.0   # half decades above take the single-query alpha in batches
BATCH_SEED = 1503


def table1() -> dict[int, int]:
    """pi(10^n) of the paper's Table 1 (tests/golden/paper_pi_pow10.txt)."""
    path = os.path.join(os.path.dirname(HERE), "tests", "golden", "paper_pi_pow10.txt")
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                n, v = line.split()
                out[10 ** int(n)] = int(v)
    return out


class ResultMismatch(RuntimeError):
    """A tuning candidate returned a different pi(x)."""


def candidates(log10x: float) -> list[float]:
    """alpha values worth timing at this size (small alpha at large x means a
    sieve too long to be competitive, and minutes of tuning)."""
    lo = 1 if log10x < 12 else 2 if log10x < 15 else 4 if log10x < 17 else 8
    hi = 48 if log10x < 15 else 96  # the largest alphas pay off only once the sieve is long
    return [a for a in ALPHAS if lo <= a <= hi]


def tune(lo: float = 7.0, hi: float = 19.0, reps: int = 3, log=print):
    import paper_1503_01839_amd as pc
    tab1 = table1()
    table = []
    d = lo
    while d <= hi + 1e-9:
        x = int(10 ** d)
        n = reps if d < 17 else 2
        want = [tab1.get(x)]  # pi(x): Table 1's, else the first candidate's

        def time(a, seg, wg):
            kw = dict(alpha=a, segment_kib=seg, wg_size=wg)
            rs = [pc.pi_count_ex(x, **kw) for _ in range(n + 1)]  # the first sizes the tables
            for r in rs:
                if want[0] is None:
                    want[0] = r.pi
                if r.pi != want[0]:
                    raise ResultMismatch(f"pi({x}) = {r.pi} at alpha {a}, shape ({seg}, {wg}); "
                                         f"expected {want[0]}")
            return statistics.median(r.ms_total for r in rs[1:])
        best = None
        for a in candidates(d):
            t = time(a, *SHAPES[0])
            log(f"  log10 x = {d:4.1f} alpha {a:5.1f} {SHAPES[0]}: {t:9.2f} ms", flush=True)
            if best is None or t < best[1]:
                best = (a, t, SHAPES[0])
        for shape in SHAPES[1:]:
            t = time(best[0], *shape)
            log(f"  log10 x = {d:4.1f} alpha {best[0]:5.1f} {shape}: {t:9.2f} ms", flush=True)
            if t < best[1]:
                best = (best[0], t, shape)
        table.append((d, best[0], best[1], best[2], best[0]))
        log(f"log10 x = {d:4.1f}: alpha {best[0]:5.1f} segment {best[2][0]} KiB "
            f"workgroup {best[2][1]}  {best[1]:9.2f} ms", flush=True)
        d += 0.5
    return table


def batch_queries(d: float) -> list[int]:
    """The batch a half decade is tuned on: x log-uniform in [d - 1/4, d + 1/4),
    as many as make a few tenths of a second of work."""
    import numpy as np
    n = 512 if d < 13 else 256 if d < 15.5 else 128
    rng = np.random.Generator(np.random.PCG64(BATCH_SEED + int(d * 10)))
    return [int(10 ** v) for v in rng.uniform(d - 0.25, d + 0.25, n)]


def tune_batch(table, reps: int = 2, log=print):
    """The batch alpha of every half decade in the table (see the module text)."""
    import time
    import paper_1503_01839_amd as pc
    out = []
    for d, a, t, sh, _ in table:
        if d > BATCH_HI + 1e-9:
            out.append((d, a, t, sh, a))
            continue
        xs = batch_queries(d)
        best = None
        first = None
        for ab in candidates(d):
            ref = pc.pi_count_batch(xs, alpha=ab)  # tables sized for this alpha
            if first is None:
                first = ref
            if ref != first:
                raise ResultMismatch(f"batch results at alpha {ab} differ from the first alpha's "
                                     f"(log10 x = {d})")
            ts = []
            for _ in range(reps):
                s = time.perf_counter()
                r = pc.pi_count_batch(xs, alpha=ab)
                ts.append((time.perf_counter() - s) * 1e3)
                if r != ref:
                    raise ResultMismatch("batch results changed between runs")
            tb = min(ts)
            log(f"  batch log10 x = {d:4.1f} n = {len(xs)} alpha {ab:5.1f}: {tb:9.2f} ms", flush=True)
            if best is None or tb < best[1]:
                best = (ab, tb)
        log(f"log10 x = {d:4.1f}: batch alpha {best[0]:5.1f}  {best[1]:9.2f} ms", flush=True)
        out.append((d, a, t, sh, best[0]))
    return out


def read_table(path: str = HEADER):
    """The entries of an existing header: (log10 x, alpha, ms, shape, batch alpha)."""
    import re
    rows = []
    for m in re.finditer(r"\{([\d.]+), ([\d.]+), (\d+), (\d+)(?:, ([\d.]+))?\}, // ([\d.]+) ms",
                         open(path).read()):
        a = float(m.group(2))
        rows.append((float(m.group(1)), a, float(m.group(6)), (int(m.group(3)), int(m.group(4))),
                     float(m.group(5)) if m.group(5) else a))
    return rows


def header_text(table) -> str:
    rows = "\n".join(f"    {{{d:.1f}, {a:g}, {sh[0]}, {sh[1]}, {ab:g}}}, // {t:.2f} ms"
                     for d, a, t, sh, ab in table)
    return f"""// pc_alpha_table.h -- alpha = y / icbrt(x) and the sieve shape per half decade of x, written by
// paper_1503_01839_amd/autotune.py from pi(x) timings on MI355X; the entry
// whose log10 x is nearest is used.  Regenerate with the tuner, do not edit.
#pragma once

struct pc_alpha_entry {{
    double log10x;
    double alpha;       // least time for one query
    unsigned seg_kib;   // LDS segment, KiB
    unsigned wg;        // workgroup threads
    double batch_alpha; // least time for a batch of queries of this size
}};

static const pc_alpha_entry kAlphaTable[] = {{
{rows}
}};
"""


def sweep(log10x: float, alphas, reps: int = 5, log=print):
    """pi(10^log10x) at every alpha x shape (median of reps, tables cached)."""
    import paper_1503_01839_amd as pc
    x = int(round(10 ** log10x))
    want = table1().get(x)
    for a in alphas:
        for seg, wg in SHAPES:
            kw = dict(alpha=a, segment_kib=seg, wg_size=wg)
            r = pc.pi_count_ex(x, **kw)  # tables sized for this alpha
            if want is None:
                want = r.pi
            rs = [pc.pi_count_ex(x, **kw) for _ in range(reps)]
            if any(q.pi != r.pi for q in rs) or (want is not None and r.pi != want):
                raise ResultMismatch(f"pi({x}) differs at alpha {a}, shape ({seg}, {wg})")
            t = statistics.median(q.ms_total for q in rs)
            log(f"  log10 x = {log10x:4.1f} alpha {a:5.1f} segment {seg} KiB workgroup {wg:4d}: "
                f"{t:9.2f} ms  (y = {r.y}, {r.segments} segments, pi = {r.pi})", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dry-run", action="store_true")
    ap.add_argument("--lo", type=float, default=7.0)
    ap.add_argument("--hi", type=float, default=19.0)
    ap.add_argument("--out", default=HEADER, help="where to write the header")
    ap.add_argument("--batch-only", action="store_true",
                    help="keep the single-query entries of the current header, tune the batch alphas")
    ap.add_argument("--sweep", type=float, default=None, metavar="LOG10X",
                    help="time every alpha x shape at x = 10^LOG10X and print; writes nothing")
    ap.add_argument("--alphas", default=None, help="comma-separated alphas for --sweep")
    args = ap.parse_args()
    if args.sweep is not None:
        alphas = [float(a) for a in args.alphas.split(",")] if args.alphas else candidates(args.sweep)
        sweep(args.sweep, alphas)
        return
    table = read_table() if args.batch_only else tune(args.lo, args.hi)
    table = tune_batch(table)
    text = header_text(table)
    if args.dry_run:
        print(text)
    else:
        with open(args.out, "w") as f:
            f.write(text)
        print("wrote", args.out)


if __name__ == "__main__":
    main()

"""Autotuner for the FFT-versus-dense crossover and the batch unit shape.

For short axes the whole n x n transform matrix is cheap to keep, and a pass
is a small matrix product on the matrix cores (the dense path); for longer
axes the r diagonally scaled FFTs win.  Where the crossover lies depends on
the precision and on how many lines a pass has (one line for a 1D
transform; many for 2D and 3D), so it is measured on the device, inside
persistent batches of many items (the batched and served forms):

    python -m paper_1901_07275_amd.autotune [--out FILE]

times a batch both ways over a grid of n for each (precision, regime) and
writes the largest n at which the dense path is still faster, plus the
rank split cap that gave the fastest ragged batch.  `dense_below()` reads
the table (the committed `tuning.json` beside this file unless another file
is given) and returns the plan option to use for an axis.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
GRID = [32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 512, 640, 768, 1024]
REGIMES = {"one_line": 1, "many_lines": 256}
DEFAULTS = {"fp32": {"one_line": 64, "many_lines": 64}, "fp64": {"one_line": 64, "many_lines": 64}}


def load(path: str = TABLE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {"dense_below": DEFAULTS, "max_split": 0, "source": "defaults"}


def dense_below(lines: int, prec: int, table: dict | None = None) -> int:
    """Plan option dense_below for an axis whose passes have `lines` lines."""
    t = (table or load())["dense_below"]
    key = "fp32" if prec == 1 else "fp64"
    regime = "one_line" if lines <= 1 else "many_lines"
    return int(t.get(key, DEFAULTS[key]).get(regime, 64))


def _time_batch(jt, torch, shapes, dense_below, prec, tol, reps):
    """Milliseconds per run of one persistent batch of the given item shapes
    (seven distinct (a, b) per shape, each planned once and shared)."""
    keys = [(s, i % 7) for i, s in enumerate(shapes)]
    distinct = sorted(set(keys))
    abs_ = [tuple((0.1 + 0.01 * j, -0.1 + 0.02 * (k % 5)) for k in range(len(s))) for s, j in distinct]
    planned = jt.plan_many([s for s, _ in distinct], abs_, tol, dense_below=[dense_below] * len(distinct))
    by_key = dict(zip(distinct, planned))
    plans = [by_key[k] for k in keys]
    arena = jt.PlanArena(planned, "cuda:0")
    sizes = [int(np.prod(s)) for s in shapes]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(int)
    dt = torch.float32 if prec == 1 else torch.float64
    code = jt.F32 if prec == 1 else jt.F64
    B = jt.Batch(plans, [jt.FORWARD] * len(plans), offs, offs, code, code, prec).bind("cuda:0")
    inp = torch.randn(sum(sizes), dtype=dt, device="cuda:0")
    out = torch.empty_like(inp)
    for _ in range(2):
        B.run(inp, out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        B.run(inp, out)
    e1.record(stream)
    torch.cuda.synchronize()
    del arena
    return e0.elapsed_time(e1) / reps


# dense must beat the FFT passes by this factor to count (the dense path's
# cost grows as n^2 per line, so a marginal win at one size is a loss in
# batches that mix in larger items)
MARGIN = 0.9


def crossover(jt, torch, prec: int, lines: int, tol: float, reps: int = 10, log=None) -> int:
    """Largest n of the grid at which dense passes beat FFT passes (by
    MARGIN) inside a persistent batch, returned as the dense_below threshold
    (one past it).  one line: 2048 1D items of length n; many lines: 64
    items of n x n."""
    best = 0
    for n in GRID:
        shapes = [(n,)] * 2048 if lines <= 1 else [(n, n)] * 64
        td = _time_batch(jt, torch, shapes, n + 1, prec, tol, reps)
        tf = _time_batch(jt, torch, shapes, 0, prec, tol, reps)
        if log:
            log("prec %d %s n %d: dense %.3f ms, fft %.3f ms" % (prec, "1d" if lines <= 1 else "2d", n, td, tf))
        if td < MARGIN * tf:
            best = n
        elif n >= 2 * max(best, 32):
            break
    return best + 1 if best else 0


def tune_split(jt, torch, log=None) -> int:
    """Rank split cap that gives the fastest ragged 1D batch (a sample of 256 items)."""
    import workloads

    items = workloads.batch_1d(256, seed=104)
    shapes = [(n,) for n, _, _ in items]
    plans = jt.plan_many(shapes, [(ab,) for _, ab, _ in items], 1e-7)
    arena = jt.PlanArena(plans, "cuda:0")
    sizes = [n for n, _, _ in items]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(int)
    inp = torch.randn(sum(sizes), dtype=torch.float32, device="cuda:0")
    out = torch.empty_like(inp)
    best, best_ms = 0, None
    for cap in (1, 2, 4, 8, 0):
        B = jt.Batch(plans, [jt.FORWARD] * len(plans), offs, offs, jt.F32, jt.F32, jt.PREC_FP32_BULK,
                     max_split=cap).bind("cuda:0")
        for _ in range(2):
            B.run(inp, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            B.run(inp, out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 100
        if log:
            log("max_split %d: %.3f ms" % (cap, ms))
        if best_ms is None or ms < best_ms:
            best, best_ms = cap, ms
    del arena
    return best


def main() -> int:
    import sys

    import torch

    import paper_1901_07275_amd as jt

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    table = {"dense_below": {}, "timings": "see the tuner's log", "source": "measured on %s" %
             torch.cuda.get_device_name(0)}
    for key, prec, tol in (("fp32", jt.PREC_FP32_BULK, 1e-7), ("fp64", jt.PREC_FP64, 1e-12)):
        table["dense_below"][key] = {r: crossover(jt, torch, prec, lines, tol, args.reps, log)
                                     for r, lines in REGIMES.items()}
    table["max_split"] = tune_split(jt, torch, log)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(table))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())

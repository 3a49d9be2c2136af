"""Benchmark: 2D uniform Jacobi transform, 1024 x 1024, forward + inverse.

One step = one forward and one inverse transform of a 1024 x 1024 tensor
(axis 0: (a, b) = (0.25, -0.35), axis 1: (-0.4, 0.1), low-rank tol 1e-12),
with the input already resident in HBM.  Both precisions are timed: the
plain fp64 path (the paper's arithmetic) gives `value`; the fp32-bulk path
(fp32 factors/FFTs, fp64 rank-sum accumulation) is reported beside it, each
with its rel-l2 against the oracle.  Each step is four
axis-pass launches (forward axis 1, forward axis 0, inverse axis 1,
inverse axis 0), each bracketed by HIP events on the launch stream, which
gives per-launch durations for the roofline and per-step latencies for
p50/p99.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       python bench.py --workload batched-1d|batched-2d [--count 4096] [--steps K]
The batched workloads time the persistent batch kernel (captured in a HIP
graph) on ragged batches of independent transforms; they plan every item on
the host first (untimed, several minutes for 4096 1D items).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

PEAK_FP64 = 78.6e12   # MI355X fp64 vector, FLOP/s
PEAK_FP32 = 157.3e12  # MI355X fp32 vector (packed; unpacked issue reaches half of it) and fp32 matrix, FLOP/s
PEAK_HBM = 8000.0     # MI355X HBM3E, GB/s


def axis_flops(n: int, L: int, nu0: int, rank: int, lines: int) -> float:
    """Algorithmic flops of one axis pass: per line r complex L-point FFTs
    (5 L log2 L each), the diagonal scalings and gather-accumulate (8 n per
    term) and the direct block (2 nu0 n)."""
    per_line = rank * (5.0 * L * math.log2(L) + 8.0 * n) + 2.0 * nu0 * n
    return per_line * lines


def source_hash(names) -> str:
    """sha256[:16] over the named files of the package (csrc/ unless a path is given)."""
    import hashlib

    h = hashlib.sha256()
    for name in names:
        path = os.path.join(ROOT, "paper_1901_07275_amd", name if "/" in name else os.path.join("csrc", name))
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def kernel_source_hash() -> str:
    """sha256[:16] over the sources the axis-pass kernel is built from."""
    return source_hash(("axis_pass.hip", "fft_line.h", "launch.h", "dense_pass.h", "dense_shape.h"))


def batch_source_hash() -> str:
    """sha256[:16] over what decides the batch kernel's work: its sources,
    the queue builder and the tuned crossover table."""
    return source_hash(("batch.hip", "batch.h", "queue.cpp", "fft_line.h", "dense_pass.h", "dense_shape.h",
                        "launch.h", "./tuning.json"))


def measured_batch_traffic(workload: str, items: int, dense_items: int):
    """HBM bytes per launch of the batch kernel on this batched workload from
    the committed rocprofv3 summary, or None (other workload, another
    FFT-versus-dense split of the items, or sources changed since the
    counters were taken)."""
    prof = os.path.join(ROOT, "profiles", "batch_kernel_%s_traffic.json" % workload.replace("batched-", ""))
    try:
        rec = json.load(open(prof))
    except (OSError, ValueError):
        return None
    if (rec.get("source_sha256_16") != batch_source_hash() or rec.get("items") != items
            or rec.get("dense_items") != dense_items):
        return None
    return float(rec["hbm_bytes"])


def measured_traffic(kernel_prefix: str, workload: str = "2d_n1024"):
    """HBM bytes per launch of the given kernel family on the given workload
    from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when
    the kernel source changed after the counters were taken."""
    prof = os.path.join(ROOT, "profiles", "axis_pass_%s_traffic.json" % workload)
    try:
        rec = json.load(open(prof))
        h = kernel_source_hash()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != h:
        return None
    vals = [v["hbm_bytes"] for k, v in rec["kernels"].items() if kernel_prefix in k]
    return float(np.mean(vals)) if vals else None


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def time_path(jt, torch, plan, alpha, prec, steps, warmup):
    """One step = the forward transform (axes d-1 .. 0) then the inverse of
    its result; every axis-pass launch is bracketed by HIP events on the
    launch stream."""
    dev = alpha.device
    g = torch.empty_like(alpha)
    back = torch.empty_like(alpha)
    stream = torch.cuda.current_stream(dev)
    axes = list(range(plan.d - 1, -1, -1))
    launches = [(ax, jt.FORWARD, alpha if i == 0 else g, g) for i, ax in enumerate(axes)]
    launches += [(ax, jt.INVERSE, g if i == 0 else back, back) for i, ax in enumerate(axes)]

    def step(evs):
        if evs:
            evs[0].record(stream)
        for i, (axis, d, src, dst) in enumerate(launches):
            plan.apply_axis(axis, d, src, dst, prec=prec, stream=stream)
            if evs:
                evs[i + 1].record(stream)
        return evs

    # every event exists before the timed region (creating them inside it
    # can stall the queue while the runtime grows its event pool)
    all_evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(launches) + 1)] for _ in range(steps)]
    for evs in all_evs:  # torch creates the device event at its first record
        for e in evs:
            e.record(stream)
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for evs in all_evs:
        step(evs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms, launch_ms = [], [[] for _ in launches]
    for evs in all_evs:
        step_ms.append(evs[0].elapsed_time(evs[-1]))
        for i in range(len(launches)):
            launch_ms[i].append(evs[i].elapsed_time(evs[i + 1]))
    return wall, step_ms, launch_ms, g, back


def cpu_cores() -> int:
    try:
        from threadpoolctl import threadpool_info

        return int(max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count() or 1]))
    except Exception:
        return os.cpu_count() or 1


def oracle_rate(fn, seconds: float) -> tuple:
    """Repeat fn() for about `seconds`; returns (repetitions, seconds used)."""
    reps, t_used = 0, 0.0
    t0 = time.perf_counter()
    while t_used < seconds or reps == 0:
        fn()
        reps += 1
        t_used = time.perf_counter() - t0
    return reps, t_used


def workload_3d(args) -> int:
    """The 3D 256^3 transform, (a, b) = (0.3, 0.3) on every axis, tol 1e-7,
    fp32 bulk (fp64 beside it): one step is a forward and an inverse
    transform, six axis-pass launches."""
    import torch

    import oracle
    import paper_1901_07275_amd as jt

    cfg = workloads.C3
    dev = torch.device("cuda:0")
    t_plan = time.perf_counter()
    plan = jt.Plan(cfg["n"], cfg["ab"], cfg["tol"]).bind(dev)
    t_plan = time.perf_counter() - t_plan
    infos = [plan.info(i) for i in range(plan.d)]
    al_np = workloads.config_input(cfg)
    alpha = torch.from_numpy(al_np).to(dev)
    coeffs = int(np.prod(cfg["n"]))
    g_ref = oracle.forward(al_np, cfg["ab"])
    res = {}
    for name, prec in (("fp32", jt.PREC_FP32_BULK), ("fp64", jt.PREC_FP64)):
        wall, step_ms, launch_ms, g, back = time_path(jt, torch, plan, alpha, prec, args.steps, args.warmup)
        ms = float(np.mean(step_ms))
        axes = list(range(plan.d - 1, -1, -1)) * 2
        flops = [axis_flops(infos[a]["n"], infos[a]["L"], infos[a]["nu0"], infos[a]["rank"], coeffs // infos[a]["n"])
                 for a in axes]
        lm = [float(np.mean(x)) for x in launch_ms]
        peak = PEAK_FP32 if name == "fp32" else PEAK_FP64
        ach = float(np.mean(flops)) / (float(np.mean(lm)) * 1e-3) / 1e12
        gg, bb = g.cpu().numpy(), back.cpu().numpy()
        res[name] = {"ms_per_step": ms, "p50_ms": percentile(step_ms, 50), "p99_ms": percentile(step_ms, 99),
                     "value": 2.0 * coeffs / (ms * 1e-3), "launch_ms": lm,
                     "rel_l2_forward": float(np.linalg.norm(gg - g_ref) / np.linalg.norm(g_ref)),
                     "rel_l2_roundtrip": float(np.linalg.norm(bb - al_np) / np.linalg.norm(al_np)),
                     "roofline": {"bound": "alu", "achieved": ach, "peak": peak / 1e12, "unit": "TFLOP/s",
                                  "frac": ach / (peak / 1e12),
                                  "traffic": measured_traffic("axis_pass<%s, 8" % ("float" if name == "fp32"
                                                                                   else "double"), "3d_n256"),
                                  "kernel": "axis_pass<%s,8>" % ("float" if name == "fp32" else "double"),
                                  "flops_per_launch": float(np.mean(flops))}}
    cpu = None
    if not args.no_cpu_baseline:
        reps, t_used = oracle_rate(lambda: oracle.inverse(oracle.forward(al_np, cfg["ab"]), cfg["ab"]),
                                   args.cpu_seconds)
        cpu = {"value": 2.0 * coeffs * reps / t_used, "unit": "coeffs/s", "cores": cpu_cores(), "kind": "oracle",
               "sample": "%d forward+inverse passes of the full 256^3 workload (dense oracle matrices along "
                         "each axis, fp64), %.1f s" % (reps, t_used)}
    head = res["fp32"]
    line = {"metric": "coeffs/s, 3D n=256 Jacobi transform, FP32 bulk (FP64 beside it) at stated rel-l2",
            "value": head["value"], "unit": "coeffs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "3d_n256_forward_plus_inverse", "n": list(cfg["n"]),
                       "ab": [list(p) for p in cfg["ab"]], "tol": cfg["tol"], "ranks": [i["rank"] for i in infos],
                       "plan_seconds": t_plan, "step": "one forward + one inverse transform (6 axis-pass launches)"},
            "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "rel_l2_forward": head["rel_l2_forward"],
            "rel_l2_roundtrip": head["rel_l2_roundtrip"], "roofline": head["roofline"], "cpu_baseline": cpu,
            "fp32": head, "fp64": res["fp64"]}
    print(json.dumps(line))
    return 0


def workload_1d(args) -> int:
    """One 1D transform of n = 1024 ((a, b) = (0.25, -0.35), tol 1e-12):
    per-launch latency over `steps` forward launches, eager and replayed
    from a captured HIP graph, fp64 and fp32 bulk."""
    import torch

    import oracle
    import paper_1901_07275_amd as jt

    cfg = workloads.C1
    dev = torch.device("cuda:0")
    plan = jt.Plan(cfg["n"], cfg["ab"], cfg["tol"]).bind(dev)
    info = plan.info(0)
    al_np = workloads.config_input(cfg)
    alpha = torch.from_numpy(al_np).to(dev)
    n = cfg["n"][0]
    g_ref = oracle.forward(al_np, cfg["ab"])
    stream = torch.cuda.current_stream(dev)
    res = {}
    for name, prec in (("fp64", jt.PREC_FP64), ("fp32", jt.PREC_FP32_BULK)):
        out = torch.empty_like(alpha)
        for _ in range(args.warmup):
            plan.forward(alpha, out, prec=prec)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for e0, e1 in evs:  # created at the first record, outside the timed launches
            e0.record(stream)
            e1.record(stream)
        torch.cuda.synchronize()
        for e0, e1 in evs:
            e0.record(stream)
            plan.forward(alpha, out, prec=prec)
            e1.record(stream)
        torch.cuda.synchronize()
        eager = [a.elapsed_time(b) for a, b in evs]
        eager_out = out.cpu().numpy()
        # the same launch captured once and replayed
        gout = torch.empty_like(alpha)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.forward(alpha, gout, prec=prec)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for e0, e1 in evs:
            e0.record(stream)
            e1.record(stream)
        torch.cuda.synchronize()
        for e0, e1 in evs:
            e0.record(stream)
            graph.replay()
            e1.record(stream)
        torch.cuda.synchronize()
        replay = [a.elapsed_time(b) for a, b in evs]
        assert np.array_equal(gout.cpu().numpy(), eager_out), "graph replay differs from the eager launch"
        ms = float(np.mean(eager))
        nbytes = (16.0 if name == "fp64" else 8.0) * info["rank"] * (n + info["L"]) \
            + (8.0 if name == "fp64" else 4.0) * info["nu0"] * n + 4.0 * n + 16.0 * n
        res[name] = {"value": n / (ms * 1e-3), "mean_ms": ms, "p50_ms": percentile(eager, 50),
                     "p99_ms": percentile(eager, 99), "graph_mean_ms": float(np.mean(replay)),
                     "graph_p50_ms": percentile(replay, 50), "graph_p99_ms": percentile(replay, 99),
                     "rel_l2_forward": float(np.linalg.norm(eager_out - g_ref) / np.linalg.norm(g_ref)),
                     "bytes_per_launch": nbytes, "hbm_gbs": nbytes / (ms * 1e-3) / 1e9}
        del graph
    head = res["fp64"]
    cpu = None
    if not args.no_cpu_baseline:
        reps, t_used = oracle_rate(lambda: oracle.forward(al_np, cfg["ab"]), min(args.cpu_seconds, 5.0))
        cpu = {"value": n * reps / t_used, "unit": "coeffs/s", "cores": cpu_cores(), "kind": "oracle",
               "sample": "%d forward transforms of the 1D n=1024 workload (dense oracle matrix built and "
                         "applied each time, fp64), %.1f s" % (reps, t_used)}
    line = {"metric": "coeffs/s and p50/p99 launch latency, one 1D n=1024 transform (plain FP64; FP32 bulk beside)",
            "value": head["value"], "unit": "coeffs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": head["mean_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "1d_n1024_forward", "n": list(cfg["n"]), "ab": [list(p) for p in cfg["ab"]],
                       "tol": cfg["tol"], "rank": info["rank"], "L": info["L"],
                       "step": "one forward transform (1 axis-pass launch)"},
            "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "rel_l2_forward": head["rel_l2_forward"],
            "roofline": {"bound": "hbm", "achieved": head["hbm_gbs"], "peak": 8000.0, "unit": "GB/s",
                         "frac": head["hbm_gbs"] / 8000.0,
                         "traffic": measured_traffic("axis_pass<double, 10, 1, 1", "1d_n1024"),
                         "kernel": "axis_pass<double,10,1,1>",
                         "bytes_per_launch": head["bytes_per_launch"],
                         "note": "a single line: launch latency, not bandwidth, bounds it"},
            "cpu_baseline": cpu, "fp64": head, "fp32": res["fp32"]}
    print(json.dumps(line))
    return 0


def factor_bytes_fp32(info: dict, lines: int) -> float:
    """Algorithmic HBM bytes of one fp32-bulk axis pass: the factors once
    (u: r n, v: r L complex; direct block nu0 n; bins n; twiddles L) plus the
    line data read and written once at the I/O dtype (counted by the caller)."""
    n, L, r, nu0 = info["n"], info["L"], info["rank"], info["nu0"]
    return 8.0 * r * n + 8.0 * r * L + 4.0 * nu0 * n + 4.0 * n + 8.0 * L


def batched(args) -> int:
    """The ragged batched form: `count` independent transforms in one
    persistent launch (captured in a HIP graph), fp32 bulk, fp32 I/O."""
    import torch

    import paper_1901_07275_amd as jt

    dev = torch.device("cuda:0")
    if args.workload == "batched-1d":
        items = workloads.batch_1d(args.count, seed=104)
        shapes = [(n,) for n, _, _ in items]
        abs_ = [(ab,) for _, ab, _ in items]
    else:
        items = workloads.batch_2d(args.count, seed=1041)
        shapes = [n for n, _, _ in items]
        abs_ = [ab for _, ab, _ in items]
    xs = [x for _, _, x in items]
    from paper_1901_07275_amd import autotune

    tuning = autotune.load()
    # the tuned FFT-versus-dense crossover: 1D items are single lines, 2D items many
    db = [autotune.dense_below(1 if len(s) == 1 else min(s), jt.PREC_FP32_BULK, tuning) for s in shapes]
    if args.dense_below >= 0:
        db = [args.dense_below] * len(shapes)
    print("planning %d items" % len(items), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plans = []
    for c0 in range(0, len(shapes), 256):  # in chunks, with a progress line each
        plans += jt.plan_many(shapes[c0:c0 + 256], abs_[c0:c0 + 256], 1e-7, dense_below=db[c0:c0 + 256])
        print("  %d planned (%.1f s)" % (len(plans), time.perf_counter() - t0), file=sys.stderr, flush=True)
    t_plan = time.perf_counter() - t0
    print("planned in %.1f s" % t_plan, file=sys.stderr, flush=True)
    arena = jt.PlanArena(plans, dev)
    sizes = [int(np.prod(s)) for s in shapes]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(int)
    coeffs = int(sum(sizes))
    B = jt.Batch(plans, [jt.FORWARD] * len(plans), offs, offs, jt.F32, jt.F32, jt.PREC_FP32_BULK,
                 max_split=int(tuning.get("max_split", 0))).bind(dev)
    inp = torch.from_numpy(np.concatenate([x.ravel() for x in xs])).to(dev, torch.float32)
    out = torch.empty_like(inp)
    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        B.run(inp, out)
    torch.cuda.synchronize()
    assert B.errors() == 0
    B.capture(inp, out)
    ms = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        B.replay(stream)
        e1.record(stream)
        ms.append((e0, e1))
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in ms]
    t_ms = float(np.mean(ms))
    # algorithmic work: every pass streams its factors (or its dense matrix)
    # once and its lines in and out (fp32); FFT passes do axis_flops on the
    # vector units, dense passes 2 n^2 flops per line on the matrix cores
    nbytes = fft_flops = mfma_flops = 0.0
    for p, s in zip(plans, shapes):
        total = int(np.prod(s))
        for ax in range(p.d):
            inf = p.info(ax)
            lines = total // inf["n"]
            if inf["nu0"] == inf["n"]:
                nbytes += 4.0 * inf["n"] * inf["n"] + 8.0 * total
                mfma_flops += 2.0 * inf["n"] * inf["n"] * lines
            else:
                nbytes += factor_bytes_fp32(inf, lines) + 8.0 * total
                fft_flops += axis_flops(inf["n"], inf["L"], inf["nu0"], inf["rank"], lines)
    t_s = t_ms * 1e-3
    # the binding roofline is the one whose peak-rate time is longest
    times = {"hbm": nbytes / (PEAK_HBM * 1e9), "mfma": mfma_flops / PEAK_FP32, "alu": fft_flops / PEAK_FP32}
    bound = max(times, key=times.get)
    fracs = {"hbm": nbytes / t_s / (PEAK_HBM * 1e9), "mfma": mfma_flops / t_s / PEAK_FP32,
             "alu": fft_flops / t_s / PEAK_FP32}
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": nbytes / t_s / 1e9, "peak": PEAK_HBM, "unit": "GB/s"}
    else:
        fl = mfma_flops if bound == "mfma" else fft_flops
        roof = {"bound": bound, "achieved": fl / t_s / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    # accuracy on a sample of items against the oracle (outside the timed region)
    import oracle

    got = out.double().cpu().numpy()
    rng = np.random.default_rng(3)
    small = [i for i, sz in enumerate(sizes) if sz <= 4096 * 8]
    errs = []
    for i in rng.choice(small, size=min(16, len(small)), replace=False):
        x32 = xs[i].astype(np.float32).astype(np.float64)
        ref = oracle.forward(x32, abs_[i])
        g = got[offs[i]:offs[i] + sizes[i]].reshape(shapes[i])
        errs.append(float(np.linalg.norm(g - ref) / np.linalg.norm(ref)))
    # the plain fp64 path on the same GPU: the same items one transform at a
    # time (items it supports: n <= 8192 per axis), and the batch restricted
    # to those items for a like-for-like ratio
    sel = [i for i, s in enumerate(shapes) if max(s) <= 8192] if not args.no_fp64_compare else []
    dev_x = [torch.from_numpy(xs[i]).to(dev) for i in sel]
    dev_g = [torch.empty_like(x) for x in dev_x]
    for i, x, g in zip(sel, dev_x, dev_g):
        plans[i].forward(x, g, prec=jt.PREC_FP64)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i, x, g in zip(sel, dev_x, dev_g):
        plans[i].forward(x, g, prec=jt.PREC_FP64)
    e1.record(stream)
    torch.cuda.synchronize()
    t64 = e0.elapsed_time(e1) if sel else float("nan")
    coeffs_sel = int(sum(sizes[i] for i in sel))
    info = B.info()
    dense_items = int(sum(1 for p in plans if p.info(0)["nu0"] == p.info(0)["n"]))
    line = {
        "metric": "coeffs/s, ragged batch of %d independent %s transforms in one persistent launch"
                  % (len(items), "1D" if args.workload == "batched-1d" else "2D"),
        "value": coeffs / (t_ms * 1e-3), "unit": "coeffs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_ms, "p50_ms": percentile(ms, 50), "p99_ms": percentile(ms, 99),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "items": len(items), "coeffs": coeffs, "tol": 1e-7,
                   "units": info["units"], "grid": info["grid"], "threads": info["threads"],
                   "plan_seconds": t_plan, "graph": True, "tuning": tuning.get("source"),
                   "dense_items": dense_items},
        "roofline": dict(roof, traffic=measured_batch_traffic(args.workload, len(items), dense_items),
                         kernel="batch_kernel<float>", bytes_per_launch=nbytes, fft_flops_per_launch=fft_flops,
                         mfma_flops_per_launch=mfma_flops, fracs=fracs,
                         peak_times_ms={k: v * 1e3 for k, v in times.items()}),
        "sample_rel_l2_max": max(errs) if errs else None,
        "fp64_one_at_a_time": ({"ms": t64, "value": coeffs_sel / (t64 * 1e-3), "items": len(sel),
                                "launches": int(sum(len(shapes[i]) for i in sel))} if sel else None),
    }
    print(json.dumps(line))
    del arena
    return 0


class PinnedPool:
    """First-fit allocator over one pinned host buffer (float32 elements), so
    that request inputs and outputs can be copied asynchronously."""

    def __init__(self, torch, elems: int):
        self.buf = torch.empty(elems, dtype=torch.float32, pin_memory=True).numpy()
        self.free = [(0, elems)]

    def alloc(self, n: int):
        for i, (o, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, sz - n)
                return o
        return None

    def release(self, o: int, n: int):
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for a, b in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + b)
            else:
                merged.append((a, b))
        self.free = merged


def serve_stream(jt, S, reqs, data, arrivals, pool):
    """Submit `reqs` to server S at the given arrival times (None: all at
    once), wait for all, return (wall seconds, per-request infos, stats delta)."""
    import threading

    before = S.stats()
    pending = []
    lock = threading.Condition()
    infos = [None] * len(reqs)
    done_count = [0]

    def waiter():
        k = 0
        while k < len(reqs):
            with lock:
                while k >= len(pending):
                    lock.wait()
                t, i, oi, oo, n = pending[k]
            infos[i] = S.wait(t)
            with lock:
                pool.release(oi, n)
                pool.release(oo, n)
                done_count[0] += 1
                lock.notify_all()
            k += 1

    th = threading.Thread(target=waiter)
    th.start()
    t0 = jt.clock()
    for i, (d, shape, ab, direction) in enumerate(reqs):
        if arrivals is not None:
            delay = t0 + arrivals[i] - jt.clock()
            if delay > 0:
                time.sleep(delay)
        n = int(np.prod(shape))
        with lock:
            while True:
                oi = pool.alloc(n)
                oo = pool.alloc(n) if oi is not None else None
                if oo is not None:
                    break
                if oi is not None:
                    pool.release(oi, n)
                lock.wait()
        x = pool.buf[oi:oi + n].reshape(shape)
        off = (i * 7919) % (len(data) - n)
        x[...] = data[off:off + n].reshape(shape)
        out = pool.buf[oo:oo + n].reshape(shape)
        t = S.submit(x, out, ab, direction)
        with lock:
            pending.append((t, i, oi, oo, n))
            lock.notify_all()
    th.join()
    wall = jt.clock() - t0
    after = S.stats()
    stats = {k: (after[k] - before[k]) if k in ("plan_hits", "plan_misses", "launches", "completed", "failed",
                                                    "plans_evicted") else after[k] for k in after}
    return wall, infos, stats


def serving(args) -> int:
    """The mixed serving stream: continuous batching with plan caching and
    HBM-footprint admission; p50/p99 latency (submit to output on the host)
    at offered loads below saturation, against the fp64 single-transform path."""
    import torch

    import paper_1901_07275_amd as jt

    reqs_all = workloads.serving_stream(args.count + args.warm, seed=105)
    warm, reqs = reqs_all[:args.warm], reqs_all[args.warm:]
    data = np.random.default_rng(107).standard_normal(1 << 25).astype(np.float32)
    pool = PinnedPool(torch, 1 << 29)  # 2 GiB of pinned host buffers
    arena = 16 << 30
    from paper_1901_07275_amd import autotune

    db = args.dense_below if args.dense_below >= 0 else autotune.dense_below(64, jt.PREC_FP32_BULK)
    db1 = args.dense_below_1d if args.dense_below_1d >= 0 else autotune.dense_below(1, jt.PREC_FP32_BULK)
    S = jt.Server(arena, tol=1e-7, prec=jt.PREC_FP32_BULK, dtype=jt.F32, dense_below=db, dense_below_1d=db1)
    print("warm-up %d requests" % len(warm), file=sys.stderr, flush=True)
    serve_stream(jt, S, warm, data, None, pool)
    # first pass over the measured requests, all offered at once: their plans
    # are mostly cold (built on the host while the stream runs)
    print("cold saturation run", file=sys.stderr, flush=True)
    wall_c, infos_c, st_c = serve_stream(jt, S, reqs, data, None, pool)
    lat_c = np.array([i["t_done"] - i["t_submit"] for i in infos_c])
    cold_c = np.array([i["cold"] for i in infos_c], dtype=bool)
    plan_s = np.array([i["plan_seconds"] for i in infos_c])
    # warm saturation: the same requests again, plans cached
    print("warm saturation run", file=sys.stderr, flush=True)
    wall, infos, st = serve_stream(jt, S, reqs, data, None, pool)
    coeffs = float(sum(int(np.prod(r[1])) for r in reqs))
    sat_rps = len(reqs) / wall
    runs = []
    for frac in args.rates:
        rate = frac * sat_rps
        arr = workloads.poisson_arrivals(len(reqs), rate, seed=106)
        print("rate %.2f x saturation (%.1f req/s)" % (frac, rate), file=sys.stderr, flush=True)
        w, inf, stt = serve_stream(jt, S, reqs, data, arr, pool)
        lat = np.array([i["t_done"] - i["t_submit"] for i in inf])
        runs.append({"load": frac, "rate_rps": rate, "wall_s": w, "coeffs_per_s": coeffs / w,
                     "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                     "plan_hit_rate": stt["plan_hits"] / max(1, stt["plan_hits"] + stt["plan_misses"]),
                     "launches": stt["launches"], "arena_peak_bytes": stt["arena_peak"]})
    S.close()
    # the plain fp64 path on the same GPU: the same requests, one at a time,
    # plans built beforehand (planning excluded), host in -> host out
    dev = torch.device("cuda:0")
    sub = reqs[:args.fp64_count]
    plans = jt.plan_many([r[1] for r in sub], [r[2] for r in sub], 1e-7)
    lat64 = []
    t0 = time.perf_counter()
    for (d, shape, ab, direction), p in zip(sub, plans):
        p.bind(dev)
        n = int(np.prod(shape))
        x = data[:n].astype(np.float64).reshape(shape)
        t1 = time.perf_counter()
        xt = torch.from_numpy(x).to(dev)
        g = p.forward(xt, prec=jt.PREC_FP64) if direction == 0 else p.inverse(xt, prec=jt.PREC_FP64)
        g.cpu()
        lat64.append(time.perf_counter() - t1)
    t64 = time.perf_counter() - t0
    c64 = float(sum(int(np.prod(r[1])) for r in sub))
    best = max(runs, key=lambda r: r["coeffs_per_s"]) if runs else None
    line = {
        "metric": "coeffs/s and p50/p99 latency, mixed serving stream (d = 1/2/3) with continuous batching",
        "value": coeffs / wall, "unit": "coeffs/s", "n_gpus": 1, "steps": len(reqs), "warmup": len(warm),
        "ms_per_step": wall / len(reqs) * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving", "requests": len(reqs), "coeffs": coeffs, "tol": 1e-7,
                   "dense_below": db, "dense_below_1d": db1,
                   "arena_bytes": arena, "warm_saturation_rps": sat_rps, "warm_saturation_launches": st["launches"]},
        "cold_pass": {"wall_s": wall_c, "coeffs_per_s": coeffs / wall_c,
                      "plan_hit_rate": st_c["plan_hits"] / max(1, st_c["plan_hits"] + st_c["plan_misses"]),
                      "cold_fraction": float(cold_c.mean()),
                      "cold_p50_ms": float(np.percentile(lat_c[cold_c], 50) * 1e3) if cold_c.any() else None,
                      "warm_p50_ms": float(np.percentile(lat_c[~cold_c], 50) * 1e3) if (~cold_c).any() else None,
                      "plan_seconds_p50": float(np.percentile(plan_s[cold_c], 50)) if cold_c.any() else None},
        "loads": runs,
        "fp64_one_at_a_time": {"requests": len(sub), "coeffs_per_s": c64 / t64,
                               "p50_ms": float(np.percentile(lat64, 50) * 1e3),
                               "p99_ms": float(np.percentile(lat64, 99) * 1e3),
                               "note": "plans prebuilt; host fp64 in and out"},
    }
    if best is not None:
        line["p50_ms"], line["p99_ms"] = best["p50_ms"], best["p99_ms"]
    print(json.dumps(line))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--warm", type=int, default=200, help="serving: warm-up requests")
    ap.add_argument("--rates", type=lambda v: [float(x) for x in v.split(",")], default=[0.5, 0.8, 0.95],
                    help="serving: offered loads as fractions of the measured saturation rate")
    ap.add_argument("--fp64-count", type=int, default=200, help="serving: requests timed on the fp64 path")
    ap.add_argument("--workload", default="2d", choices=["2d", "1d", "3d", "batched-1d", "batched-2d", "serving"],
                    help="2d: the 1024 x 1024 forward + inverse headline; 1d: launch latency of one n = 1024 "
                         "transform; 3d: the 256^3 transform; batched-*: ragged batches; serving: request stream")
    ap.add_argument("--count", type=int, default=4096, help="items of a batched workload (serving: requests)")
    ap.add_argument("--dense-below", type=int, default=-1,
                    help="batched/serving: dense-path threshold instead of the tuned one (1: FFT everywhere)")
    ap.add_argument("--dense-below-1d", type=int, default=-1,
                    help="serving: the same for 1D requests")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="batched: skip the one-at-a-time fp64 comparison (for profiler runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), to calibrate "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE against known bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(one GPU's share of the work is the whole workload); run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    if args.copy_probe:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "launches": 5}))
        return 0

    if args.workload == "serving":
        return serving(args)
    if args.workload == "3d":
        return workload_3d(args)
    if args.workload == "1d":
        return workload_1d(args)
    if args.workload != "2d":
        return batched(args)

    import paper_1901_07275_amd as jt

    cfg = workloads.C2
    dev = torch.device("cuda:0")
    t_plan = time.perf_counter()
    plan = jt.Plan(cfg["n"], cfg["ab"], cfg["tol"]).bind(dev)
    t_plan = time.perf_counter() - t_plan
    infos = [plan.info(i) for i in range(plan.d)]
    al_np = workloads.config_input(cfg)
    alpha = torch.from_numpy(al_np).to(dev)
    n0, n1 = cfg["n"]
    coeffs = n0 * n1

    results = {}
    for name, prec in (("fp64", jt.PREC_FP64), ("fp32", jt.PREC_FP32_BULK)):
        wall, step_ms, launch_ms, g, back = time_path(jt, torch, plan, alpha, prec, args.steps, args.warmup)
        ms = float(np.mean(step_ms))
        flops = [axis_flops(infos[1]["n"], infos[1]["L"], infos[1]["nu0"], infos[1]["rank"], n0),
                 axis_flops(infos[0]["n"], infos[0]["L"], infos[0]["nu0"], infos[0]["rank"], n1)]
        launch_avg = [float(np.mean(x)) for x in launch_ms]
        launch_flops = [flops[0], flops[1], flops[0], flops[1]]
        results[name] = dict(ms_per_step=ms, p50_ms=percentile(step_ms, 50), p99_ms=percentile(step_ms, 99),
                             wall_s=wall, value=2.0 * coeffs / (ms * 1e-3),
                             launch_ms=launch_avg, launch_flops=launch_flops,
                             g=g.cpu().numpy(), back=back.cpu().numpy())

    # accuracy against the oracle (outside the timed region)
    import oracle

    g_ref = oracle.forward(al_np, cfg["ab"])
    for name in results:
        r = results[name]
        r["rel_l2_forward"] = float(np.linalg.norm(r["g"] - g_ref) / np.linalg.norm(g_ref))
        r["rel_l2_roundtrip"] = float(np.linalg.norm(r["back"] - al_np) / np.linalg.norm(al_np))
        del r["g"], r["back"]

    # roofline of the dominant kernel (the axis pass) for each path; the
    # headline is the fp64 path
    def roofline(r, peak, kernel, prefix):
        launch_ms = float(np.mean(r["launch_ms"]))
        launch_flops = float(np.mean(r["launch_flops"]))
        achieved = launch_flops / (launch_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": achieved, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / (peak / 1e12), "traffic": measured_traffic(prefix), "kernel": kernel,
                "launch_ms": launch_ms, "flops_per_launch": launch_flops}

    head = results["fp64"]
    roof = roofline(head, PEAK_FP64, "axis_pass<double,10>", "axis_pass<double, 10")
    results["fp32"]["roofline"] = roofline(results["fp32"], PEAK_FP32, "axis_pass<float,10>",
                                           "axis_pass<float, 10")

    cpu = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        def oracle_step():
            gg = oracle.forward(al_np, cfg["ab"])
            oracle.inverse(gg, cfg["ab"])

        reps, t_used = oracle_rate(oracle_step, args.cpu_seconds)
        with threadpool_limits(limits=1):
            reps1, t1 = oracle_rate(oracle_step, args.cpu_seconds / 2)
        cpu = {"value": 2.0 * coeffs * reps / t_used, "unit": "coeffs/s", "cores": cpu_cores(), "kind": "oracle",
               "sample": "%d forward+inverse passes of the full 1024x1024 workload (dense oracle matrices "
                         "applied along each axis in fp64, numpy/BLAS on all host threads), %.1f s"
                         % (reps, t_used),
               "single_thread": {"value": 2.0 * coeffs * reps1 / t1, "unit": "coeffs/s", "cores": 1,
                                 "sample": "%d passes with BLAS held to one thread, %.1f s" % (reps1, t1)}}

    line = {
        "metric": "coeffs/s, 2D n=1024 Jacobi FP32 vs FP64 at stated rel-l2; p50/p99 latency",
        "value": head["value"],
        "unit": "coeffs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2d_n1024_forward_plus_inverse", "n": list(cfg["n"]),
                   "ab": [list(p) for p in cfg["ab"]], "tol": cfg["tol"],
                   "ranks": [i["rank"] for i in infos], "plan_seconds": t_plan,
                   "step": "one forward + one inverse transform (4 axis-pass launches)"},
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "rel_l2_forward": head["rel_l2_forward"],
        "rel_l2_roundtrip": head["rel_l2_roundtrip"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64": {k: v for k, v in results["fp64"].items()},
        "fp32": results["fp32"],
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())

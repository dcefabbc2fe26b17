#!/usr/bin/env python3
"""Benchmark: all pairs of geodesic distances on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Workloads (synthetic inputs from ``synth``; the paper's own images are not
available):
  blob128    (default) 128x128 blob image, 4-neighbours, w = f(p)+f(q):
             a step is one all-pairs call of the filling-rate method
             (Section 3.4), 16384^2 int32 = 1 GiB; the naive method (one
             propagation per pixel) is timed beside it on the same image
  uniform32  32x32 iid image, naive method (4 MiB output)
  voronoi192 192x192x8 Voronoi image, w = 1 + L1, filling-rate vs naive (5.4 GB)
  batched    256 iid images of sides 24..96 in one call, both methods
  serve      Poisson request stream through the continuous-batching server
  hbmcopy    a plain 1 GiB device copy (calibrates rocprofv3's byte counters)
  blob128c8  the 128x128 blob image with 8-neighbours, filling-rate vs naive
  deltar     the paper's method comparison (Sections 3 and 4): propagations
             to fill D for naive, spiral, spiral with repulsion 3, geodesic
             extrema and filling rate, 8-neighbours, on 25x25 stand-ins for
             "random", "bumps" and "hairpin bend" (spiral methods averaged
             over --draw-seeds draw sequences), with filling-rate curves;
             then every tree method timed once on the 128x128 blob image
  graph      a random geometric graph (CSR, 4096 vertices, 6 nearest
             neighbours + an x-ordered chain, Euclidean integer weights):
             filling-rate vs naive through the general-graph path (Section 5)

Prints ONE JSON line.  Inputs are resident on the GPU when the timed region
starts; the timed region is bracketed by torch.cuda.synchronize().
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "distance entries/sec and HBM GB/s fraction, tree_fill vs naive GPU; p50/p99 latency"
HBM_PEAK_GBPS = 8000.0            # MI355X HBM3E, published
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # 256 CUs x 64 int32 lanes/clk x 2.4 GHz = 39.3 Tops/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


# ---------------------------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on a bounded sample of the same workload.
# ---------------------------------------------------------------------------------------------
def cpu_baseline_fr(img, conn, n_prop_total, budget_s):
    import oracle
    N = img.shape[0] * img.shape[1]
    t0 = time.perf_counter()
    oracle.extrema(img, conn=conn)
    t_setup = time.perf_counter() - t0
    probe = 8
    t0 = time.perf_counter()
    oracle.filling_rate(img, conn=conn, max_steps=probe)
    t_probe = time.perf_counter() - t0
    per = max((t_probe - t_setup) / probe, 1e-6)
    steps = int(max(probe, min(n_prop_total, (budget_s - t_setup) / per)))
    for _ in range(3):
        t0 = time.perf_counter()
        fr = oracle.filling_rate(img, conn=conn, max_steps=steps)
        t = time.perf_counter() - t0
        per = (t - t_setup) / max(fr.n_prop, 1)
        if t > 0.6 * budget_s or steps >= n_prop_total:
            break
        steps = int(min(n_prop_total, steps * budget_s / max(t, 1e-3)))
    t_total = t_setup + per * n_prop_total
    return {"value": N * N / t_total, "unit": "distance entries/s", "cores": 1, "kind": "oracle",
            "sample": f"first {fr.n_prop} of {n_prop_total} filling-rate steps (the loop is sequential; 1 thread); "
                      f"whole-job time extrapolated as setup + {n_prop_total} x mean step time (early steps fill "
                      f"the most pairs, so this is an upper bound of the full run)",
            "seconds_measured": round(t, 2), "seconds_extrapolated": round(t_total, 1)}


def cpu_baseline_naive(img, conn, budget_s):
    import oracle
    N = img.shape[0] * img.shape[1]
    cores = host_cores()
    rows = min(N, max(cores, 64))
    t0 = time.perf_counter()
    oracle.rows(img, np.arange(rows), conn=conn, threads=cores)
    t = time.perf_counter() - t0
    rows2 = int(min(N, max(rows, rows * budget_s / max(t, 1e-6))))
    if rows2 > rows:
        t0 = time.perf_counter()
        oracle.rows(img, np.arange(rows2), conn=conn, threads=cores)
        t = time.perf_counter() - t0
        rows = rows2
    return {"value": rows * N / t, "unit": "distance entries/s", "cores": cores, "kind": "oracle",
            "sample": f"naive method, propagations from the first {rows} of {N} sources, OpenMP over sources"}


# ---------------------------------------------------------------------------------------------
# Single-image workloads: filling rate vs naive.
# ---------------------------------------------------------------------------------------------
def run_single(args, name, img, conn, modes):
    import torch
    from paper_2007_16076_amd import gapd
    ctx = gapd.Context(img, conn=conn)
    N = ctx.N
    out = torch.empty((N, N), dtype=torch.int32, device="cuda")
    res = {}
    for mode in modes:
        stats, wall = [], []
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = ctx.all_pairs(mode, out=out)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) * 1e3
            log(f"[{name}] mode={mode} call {i}: {dt:.1f} ms (events {st.ms_total:.1f} ms) n_prop={st.n_prop}")
            if i >= args.warmup:
                stats.append(st)
                wall.append(dt)
        kstats = stats
        if mode != gapd.MODE_NAIVE:
            # one more call, outside the timed ones, with every loop launch
            # bracketed by events: the per-kernel durations of the roofline
            _, st = ctx.all_pairs(mode, out=out, time_kernels=True)
            torch.cuda.synchronize()
            kstats = [st]
        res[mode] = (stats, wall, kstats)
    return ctx, res


def roofline_hbm(bytes_per_launch, ms):
    ach = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBPS, 7), "traffic": None}


def kernels_sha256():
    """SHA-256 over the device-code sources (dev_common.h and the k_*.hip files, in name order)."""
    csrc = os.path.join(ROOT, "paper_2007_16076_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name == "dev_common.h" or (name.startswith("k_") and name.endswith(".hip")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def wall_clock_khz():
    """The device's constant clock (hipDeviceAttributeWallClockRate = 10017), in kHz."""
    import ctypes
    import torch
    try:
        lib = ctypes.CDLL("libamdhip64.so")
        v = ctypes.c_int(0)
        if lib.hipDeviceGetAttribute(ctypes.byref(v), 10017, torch.cuda.current_device()) == 0 and v.value > 0:
            return v.value
    except OSError:
        pass
    return 100000


def fill_trace(ctx, mode, out, path=None):
    """One extra call with the per-step trace of the tree modes: what each
    fill launch walked and found, and how long its blocks took.  Returns a
    summary by phase of the run; the per-step table goes to ``path``."""
    import torch
    N = ctx.N
    tr = torch.zeros(32 * N, dtype=torch.int64, device="cuda")
    _, st = ctx.all_pairs(mode, out=out, step_trace=tr)
    torch.cuda.synchronize()
    t = tr.view(N, 32)[: st.n_prop].cpu().numpy().astype(np.float64)
    us = 1e3 / wall_clock_khz()
    start = (2.0 ** 63 - 1) - t[:, 6]
    span = np.where(t[:, 11] > 0, (t[:, 7] - start) * us, 0.0)
    launch_span = np.where(t[:, 8] > 0, (np.maximum(t[:, 7], t[:, 13]) - start) * us, span)
    cols = {"visits": t[:, 0], "new_pairs": t[:, 1], "max_walk": t[:, 2], "walkers": t[:, 3],
            "fill_span_us": span, "fill_block_max_us": t[:, 4] * us,
            "fill_block_mean_us": t[:, 5] * us / np.maximum(t[:, 11], 1), "spec_pieces": t[:, 8],
            "spec_max_us": t[:, 9] * us, "select_us": t[:, 10] * us, "spec_converged": t[:, 12],
            "launch_span_us": launch_span,
            "spec_tail_us": np.where(t[:, 8] > 0, np.maximum(t[:, 13] - t[:, 7], 0.0) * us, 0.0),
            "cache_hit": t[:, 14]}
    nb = np.maximum(t[:, 11], 1)
    for i, k in enumerate(["tables", "detect", "write", "flush"]):
        cols[f"ph_{k}_us"] = t[:, 16 + i] * us / nb  # mean over the step's fill blocks
    npc = np.maximum(t[:, 8], 1)
    for i, k in ((15, "stage"), (20, "round"), (21, "store")):
        cols[f"spec_{k}_us"] = t[:, i] * us / npc  # mean over the step's pieces
    for i, k in ((24, "pass"), (25, "min"), (26, "sort"), (27, "rest")):
        cols[f"sel_{k}_us"] = t[:, i] * us
    cols["ph_detect_max_us"] = t[:, 22] * us
    cols["ph_write_max_us"] = t[:, 23] * us
    n = st.n_prop
    edges = sorted({0, min(100, n), min(1000, n), min(3000, n), min(6000, n), min(9000, n), n})
    phases = []
    for a, b in zip(edges[:-1], edges[1:]):
        if b > a:
            phases.append(dict(steps=[int(a), int(b)], **{k: round(float(v[a:b].mean()), 2) for k, v in cols.items()}))
    summary = {"n_prop": int(n), "ms_total": round(st.ms_total, 3),
               "totals": {"visits": float(t[:, 0].sum()), "new_pairs": float(t[:, 1].sum())},
               "mean": {k: round(float(v.mean()), 2) for k, v in cols.items()},
               "max": {k: round(float(v.max()), 2) for k, v in cols.items()}, "phases": phases}
    if path:
        np.savetxt(path, np.column_stack([cols[k] for k in cols]), fmt="%.3f", delimiter=",",
                   header=",".join(cols), comments="")
    return summary


def _counters(workload, kernel_prefix):
    """The committed rocprofv3 counter summary of a kernel (profiles/
    traffic_<workload>.json), or None when there is none or the kernels have
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernels_sha256") != kernels_sha256():
        return None, None
    for name, k in t["kernels"].items():
        if name.startswith(kernel_prefix):
            return t, k
    return None, None


def measured_traffic(workload, kernel_prefix):
    """HBM bytes per launch of a kernel from the counter summary (FETCH_SIZE and
    WRITE_SIZE, scaled by the plain-copy calibration), or None."""
    t, k = _counters(workload, kernel_prefix)
    if k is None or "fetch_kib" not in k:
        return None
    kib = k["fetch_kib"] * t["fetch_factor"] + k["write_kib"] * t["write_factor"]
    return round(kib * 1024 / max(k["dispatches"], 1))


def alu_side(ops_per_launch, ms, workload, kernel_prefix):
    """The ALU side of a kernel's roofline: the method's integer operations
    per launch (2 per relaxation: add and min) over the live launch duration,
    against the chip's int32 vector peak; beside it the issued VALU lane
    operations (SQ_INSTS_VALU x 64 per launch, from the counter summary of
    the same kernels) over the same duration, when there is one."""
    ach = ops_per_launch / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    d = {"bound": "alu", "achieved": round(ach, 4), "peak": round(VALU_PEAK_TOPS, 1), "unit": "Tops/s",
         "frac": round(ach / VALU_PEAK_TOPS, 6), "ops_per_launch": round(ops_per_launch)}
    _, k = _counters(workload, kernel_prefix)
    if k is not None and "valu_insts" in k and ms > 0:
        lane_ops = 64.0 * k["valu_insts"] / max(k["dispatches"], 1)
        iss = lane_ops / (ms * 1e-3) / 1e12
        d.update(issued_lane_ops_per_launch=round(lane_ops), issued_achieved=round(iss, 4),
                 issued_frac=round(iss / VALU_PEAK_TOPS, 6))
    else:
        d.update(issued_lane_ops_per_launch=None, issued_achieved=None, issued_frac=None)
    return d


def single_image_line(args, workload, img, conn, desc, fr=True):
    from paper_2007_16076_amd import gapd
    N = img.shape[0] * img.shape[1]
    E_dir = edges_directed(img.shape[0], img.shape[1], conn)
    modes = [gapd.MODE_TREE_FILL_FR, gapd.MODE_NAIVE] if fr else [gapd.MODE_NAIVE]
    ctx, res = run_single(args, workload, img, conn, modes)
    nst, nwall, _ = res[gapd.MODE_NAIVE]
    naive_ms = [s.ms_total for s in nst]
    naive_kernel_ms = float(np.mean([s.ms_kernel for s in nst]))
    naive_rounds = float(np.mean([s.rounds for s in nst])) / N
    naive = {"value": N * N / (np.mean(naive_ms) * 1e-3), "unit": "distance entries/s",
             "ms_per_call": round(float(np.mean(naive_ms)), 3), "p50_ms": round(pct(naive_ms, 50), 3),
             "p99_ms": round(pct(naive_ms, 99), 3), "kernel_ms": round(naive_kernel_ms, 3),
             "rounds_per_propagation": round(naive_rounds, 2)}
    roof_naive = roofline_hbm(4.0 * N * N, naive_kernel_ms)
    roof_naive["kernel"] = "k_relax_rows (one propagation per workgroup, writes its row of D)"
    roof_naive["algorithmic_bytes_per_launch"] = 4 * N * N
    roof_naive["traffic"] = measured_traffic(workload, "k_relax_rows<")
    naive_rounds_total = float(np.mean([s.rounds for s in nst]))
    roof_naive["alu"] = alu_side(2.0 * E_dir * naive_rounds_total, naive_kernel_ms, workload, "k_relax_rows<")
    line = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic", "config": dict(desc, workload=workload, N=N, conn=conn,
                                                output_bytes=4 * N * N)}
    if not fr:
        line.update(value=naive["value"], unit="distance entries/s", ms_per_step=naive["ms_per_call"],
                    p50_ms=naive["p50_ms"], p99_ms=naive["p99_ms"], naive=naive, roofline=roof_naive)
        line["config"]["mode"] = "naive"
        return line, ctx
    fst, fwall, kst = res[gapd.MODE_TREE_FILL_FR]
    fr_ms = [s.ms_total for s in fst]
    s0 = kst[-1]
    n_prop = s0.n_prop
    step_ms = float(s0.ms_step_kernels) / max(n_prop, 1)
    fill_ms = float(s0.ms_fill_kernels) / max(n_prop, 1)
    hits, n_spec = int(s0.n_cache_hits), int(s0.n_prop_speculative)
    spec = hits > 0 or n_spec > 0
    # rounds per propagation, over every propagation computed (setup, main
    # loop misses, speculative)
    rounds = s0.rounds / max(n_prop - hits + n_spec + 2, 1)
    # Per-launch algorithmic work:
    #   fill: the D entries and mask bits the whole run writes once, averaged
    #   per launch, plus one propagation's distances and predecessors (4N + N
    #   bytes: the tree the launch reads);
    #   ALU: 2 ops (add, min) per relaxation, |E_dir| relaxations per sweep
    #   round; the fill launch holds the speculative pieces' rounds, the step
    #   launch the rest (cache misses; the two setup propagations included).
    fill_bytes = (4.0 * N * N + N * N / 8.0) / max(n_prop, 1) + 5.0 * N
    roof_fill = roofline_hbm(fill_bytes, fill_ms)
    fill_name = "k_fr_fill_spec" if spec else "k_fr_fill"
    roof_fill.update(kernel=fill_name + " (redundancy fill along the geodesic tree"
                     + (", beside the speculative propagations)" if spec else ")"),
                     algorithmic_bytes_per_launch=round(fill_bytes), avg_launch_ms=round(fill_ms, 5),
                     traffic=measured_traffic(workload, fill_name + "<"))
    spec_rounds = int(getattr(s0, "rounds_speculative", 0))
    roof_fill["alu"] = alu_side(2.0 * E_dir * spec_rounds / max(n_prop, 1), fill_ms, workload, fill_name + "<")
    step_ops = 2.0 * E_dir * (s0.rounds - spec_rounds) / max(n_prop, 1)
    if spec:
        # With the tree cache a step launch is the select pass (count, rank or
        # distance, and cache slot: 12 bytes per point read) plus, on a miss,
        # one propagation writing N tree words.
        step_bytes = 12.0 * N + 4.0 * N * (n_prop - hits) / max(n_prop, 1)
        roof_step = roofline_hbm(step_bytes, step_ms)
        t_part, t_step = measured_traffic(workload, "k_sel_part<"), measured_traffic(workload, "k_fr_step_spec<")
        roof_step.update(kernel="k_sel_part + k_fr_step_spec (least-filled select: the pass over the points in "
                                "many workgroups, then the argmin, speculation plan and, on a cache miss, one "
                                "propagation + tree in one workgroup)",
                         algorithmic_bytes_per_launch=round(step_bytes), avg_launch_ms=round(step_ms, 5),
                         traffic=(t_part + t_step) if t_part is not None and t_step is not None else None)
        roof_step["alu"] = alu_side(step_ops, step_ms, workload, "k_fr_step_spec<")
    else:
        ach = step_ops / (step_ms * 1e-3) / 1e12
        roof_step = {"bound": "alu", "achieved": round(ach, 4), "peak": round(VALU_PEAK_TOPS, 1), "unit": "Tops/s",
                     "frac": round(ach / VALU_PEAK_TOPS, 6), "traffic": measured_traffic(workload, "k_fr_step<"),
                     "kernel": "k_fr_step (least-filled select + one propagation + tree, one workgroup)",
                     "algorithmic_ops_per_launch": round(step_ops), "avg_launch_ms": round(step_ms, 5)}
    dominant, other = (roof_step, roof_fill) if step_ms >= fill_ms else (roof_fill, roof_step)
    value = N * N / (np.mean(fr_ms) * 1e-3)
    line.update(value=value, unit="distance entries/s", ms_per_step=round(float(np.mean(fr_ms)), 3),
                p50_ms=round(pct(fr_ms, 50), 3), p99_ms=round(pct(fr_ms, 99), 3),
                n_prop=int(n_prop), n_prop_setup=int(s0.n_prop_setup),
                n_prop_speculative=n_spec, n_cache_hits=hits,
                cache_hit_rate=round(hits / max(n_prop - 1, 1), 4),
                rounds_per_propagation=round(rounds, 2), rounds_speculative=spec_rounds,
                propagation_saving_vs_naive=round(1.0 - (n_prop + s0.n_prop_setup) / N, 4),
                fr_setup_ms=round(float(np.mean([s.ms_setup for s in fst])), 3),
                fr_loop_kernel_ms={"select_propagate": round(step_ms * n_prop, 3),
                                   "fill": round(fill_ms * n_prop, 3)},
                naive=naive, fr_time_over_naive=round(float(np.mean(fr_ms)) / naive["ms_per_call"], 2),
                roofline=dominant, roofline_other=other, roofline_naive=roof_naive)
    line["config"]["mode"] = "tree_fill_filling_rate (naive timed beside it)"
    if getattr(args, "fill_trace", None):
        import torch
        out = torch.empty((N, N), dtype=torch.int32, device="cuda")
        line["fill_trace"] = fill_trace(ctx, gapd.MODE_TREE_FILL_FR, out, args.fill_trace)
    return line, ctx


def edges_directed(H, W, conn):
    e = H * (W - 1) + (H - 1) * W
    if conn == 8:
        e += 2 * (H - 1) * (W - 1)
    return 2 * e


# ---------------------------------------------------------------------------------------------
# Batched and serving workloads.
# ---------------------------------------------------------------------------------------------
def batched_line(args):
    import torch
    import synth
    from paper_2007_16076_amd import gapd
    imgs = synth.config4()
    shapes = [im.shape for im in imgs]
    offs = gapd.pack_offsets(shapes)
    total = int(offs[-1])
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    res = {}
    for mode in (gapd.MODE_NAIVE, gapd.MODE_TREE_FILL_FR):
        ws = torch.empty(gapd.batched_workspace_size(shapes, mode=mode), dtype=torch.uint8, device="cuda")
        ms = []
        steps = args.steps if mode == gapd.MODE_NAIVE else max(1, min(args.steps, 2))
        for i in range(args.warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, nprop = gapd.all_pairs_batched(imgs, mode=mode, out=out, offsets=offs, workspace=ws)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) * 1e3
            log(f"[batched] mode={mode} call {i}: {dt:.1f} ms")
            if i >= args.warmup:
                ms.append(dt)
        res[mode] = (ms, nprop)
    nms, _ = res[gapd.MODE_NAIVE]
    fms, fprop = res[gapd.MODE_TREE_FILL_FR]
    n_sum = sum(h * w for h, w in shapes)
    line = {"metric": METRIC, "value": total / (np.mean(fms) * 1e-3), "unit": "distance entries/s",
            "n_gpus": 1, "steps": len(fms), "warmup": args.warmup, "ms_per_step": round(float(np.mean(fms)), 2),
            "p50_ms": round(pct(fms, 50), 2), "p99_ms": round(pct(fms, 99), 2),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic",
            "config": {"workload": "batched256", "images": len(imgs), "sides": "24..96", "conn": 4,
                       "entries": total, "output_bytes": 4 * total, "mode": "tree_fill_filling_rate"},
            "naive": {"value": total / (np.mean(nms) * 1e-3), "ms_per_call": round(float(np.mean(nms)), 2),
                      "p50_ms": round(pct(nms, 50), 2), "p99_ms": round(pct(nms, 99), 2),
                      "hbm_gbps_output": round(4 * total / (np.mean(nms) * 1e-3) / 1e9, 1)},
            "propagation_saving_vs_naive": round(1.0 - (float(np.sum(fprop)) + 2 * len(imgs)) / n_sum, 4),
            "roofline": roofline_hbm(4.0 * total, float(np.mean(nms)))}
    line["roofline"]["kernel"] = "k_relax_rows_batched (whole naive call, output bytes only)"
    # ALU side: the sweep rounds of every image's propagations, counted by a
    # single-image naive call per image (outside the timed calls; the batched
    # kernel runs the same sweeps to the same fixed points)
    ops = 0.0
    for im in imgs:
        _, st = gapd.Context(im).all_pairs(gapd.MODE_NAIVE)
        ops += 2.0 * edges_directed(im.shape[0], im.shape[1], 4) * st.rounds
    torch.cuda.synchronize()
    line["roofline"]["alu"] = alu_side(ops, float(np.mean(nms)), "batched256", "k_relax_rows_batched<")
    return line


def serve_line(args, rate=None):
    """C5: Poisson arrivals of a 70/30 mix of all-pairs blob jobs (sides 64..192)
    and multi-source jobs on resident 512x512 blob images (K in 1..512), through
    the server.  Latency runs from each request's scheduled arrival time to its
    completion, so it includes queueing."""
    import torch
    import synth
    from paper_2007_16076_amd import gapd
    rate = args.rate if rate is None else rate
    n = args.requests
    reqs, images = synth.serving_trace(rate, n, side=(64, 192))
    free, _ = torch.cuda.mem_get_info()
    arena_bytes = int(min(200e9, free * 0.8))
    srv = gapd.Server(arena_bytes, max_slots=args.slots)
    mode = gapd.MODE_TREE_FILL_FR if args.serve_mode == "tree_fill" else gapd.MODE_NAIVE
    torch.cuda.synchronize()
    # A collector thread releases every finished job at once (its result then
    # leaves the arena), as a client that consumes results would; ctypes
    # drops the GIL inside the library calls.
    import queue
    import threading
    pending_q = queue.Queue()
    lat, lat_kind, counts = [], {"all_pairs": [], "multi_source": []}, {"entries": 0, "done": 0}

    def collect():
        pending, last_log = [], time.perf_counter()
        while counts["done"] < n:
            while True:
                try:
                    pending.append(pending_q.get_nowait())
                except queue.Empty:
                    break
            still = []
            for t, r, lag in pending:
                res = srv.poll(t)
                if res is None:
                    still.append((t, r, lag))
                    continue
                ms = (res.t_done - res.t_submit + lag) * 1e3
                lat.append(ms)
                lat_kind[r.kind].append(ms)
                counts["entries"] += res.elems
                srv.release(t)
                counts["done"] += 1
            pending = still
            if time.perf_counter() - last_log > 20:
                log(f"[serve {args.serve_mode} rate {rate}] {counts['done']}/{n} done")
                last_log = time.perf_counter()
            time.sleep(0.0005)

    th = threading.Thread(target=collect, daemon=True)
    t0 = time.perf_counter()
    th.start()
    for r in reqs:
        while True:
            wait_s = r.t_arrival - (time.perf_counter() - t0)
            if wait_s <= 0:
                break
            time.sleep(min(0.001, wait_s))
        lag = time.perf_counter() - t0 - r.t_arrival  # submitted this late after its scheduled arrival
        if r.kind == "all_pairs":
            t = srv.submit_all_pairs(images[r.image_id], mode=mode)
        else:
            t = srv.submit_multi_source(images[r.image_id], r.sources)
        pending_q.put((t, r, lag))
    th.join()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    entries = counts["entries"]
    srv.close()
    del srv
    torch.cuda.empty_cache()
    kinds = {k: {"jobs": len(v), "p50_ms": round(pct(v, 50), 2), "p99_ms": round(pct(v, 99), 2)}
             for k, v in lat_kind.items() if v}
    log(f"[serve {args.serve_mode} rate {rate}] {n} jobs in {wall:.1f} s")
    return {"metric": METRIC, "value": entries / wall, "unit": "distance entries/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": round(wall * 1e3, 1), "p50_ms": round(pct(lat, 50), 2),
            "p99_ms": round(pct(lat, 99), 2), "jobs_per_s": round(n / wall, 2), "by_kind": kinds,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": "serve", "rate_req_s": rate, "requests": n, "slots": args.slots,
                       "all_pairs_mode": args.serve_mode, "arena_bytes": arena_bytes,
                       "latency": "from the scheduled arrival to completion"}}


def hbmcopy_line(args):
    import torch
    n = 1 << 28  # int32 elements: 1 GiB
    a = torch.empty(n, dtype=torch.int32, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    ms = []
    for i in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        if i >= args.warmup:
            ms.append(e0.elapsed_time(e1))
    t = float(np.mean(ms))
    return {"metric": "HBM copy, 1 GiB read + 1 GiB written (calibration)", "value": 2 * 4 * n / (t * 1e-3) / 1e9,
            "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic", "config": {"workload": "hbmcopy", "bytes_read": 4 * n, "bytes_written": 4 * n}}


def deltar_line(args):
    """Propagation counts and relative differences of the tree methods (the
    comparison of Sections 3 and 4), all computed by the GPU library."""
    import torch
    import synth
    from paper_2007_16076_amd import gapd
    conn = 8
    out = {}
    t0 = time.time()

    def run(ctx, mode=None, draws=None, h=0):
        N = ctx.N
        fil = torch.zeros(N, dtype=torch.int64, device="cuda")
        if draws is None:
            _, st = ctx.all_pairs(mode, filled_out=fil)
        else:
            _, st = ctx.all_pairs_spiral(draws, h=h, filled_out=fil)
        torch.cuda.synchronize()
        return st, fil.cpu().numpy()[:st.n_prop]

    for name, img in synth.deltar_images().items():
        N = img.size
        A = N * (N - 1) // 2
        ctx = gapd.Context(img, conn=conn)
        res = {}
        curves = {}
        for mname, mode in (("filling_rate", gapd.MODE_TREE_FILL_FR), ("extrema", gapd.MODE_TREE_FILL_EXTREMA)):
            st, fil = run(ctx, mode=mode)
            res[mname] = {"n_prop": int(st.n_prop), "n_prop_plus_setup": int(st.n_prop + st.n_prop_setup)}
            curves[mname] = fil
        for mname, h in (("spiral", 0), ("spiral_repulsion3", 3)):
            ns = []
            for sd in range(args.draw_seeds):
                st, fil = run(ctx, draws=synth.spiral_draws(sd, N), h=h)
                ns.append(int(st.n_prop))
                if sd == 0:
                    curves[mname] = fil
            res[mname] = {"n_prop_mean": float(np.mean(ns)), "n_prop_std": round(float(np.std(ns)), 2),
                          "n_prop_min": min(ns), "n_prop_max": max(ns), "draw_seeds": args.draw_seeds}
        n_sp = res["spiral"]["n_prop_mean"]
        for mname, r in res.items():
            n = r.get("n_prop_mean", r.get("n_prop"))
            r["dr_naive_pct"] = round(100.0 * (N - n) / N, 1)
            r["dr_spiral_pct"] = round(100.0 * (n_sp - n) / n_sp, 1)
            if "n_prop_plus_setup" in r:
                r["dr_naive_plus_setup_pct"] = round(100.0 * (N - r["n_prop_plus_setup"]) / N, 1)
                r["dr_spiral_plus_setup_pct"] = round(100.0 * (n_sp - r["n_prop_plus_setup"]) / n_sp, 1)
        # filling rate tau = a / A after 10 %, 25 %, 50 % and 75 % of N propagations
        tau = {m: {f"{q}%": round(float(c[min(len(c), max(1, int(q * N / 100))) - 1]) / A, 4) for q in (10, 25, 50, 75)}
               for m, c in curves.items()}
        out[name] = {"N": N, "sha256": synth.sha256(img), "naive_n_prop": N, "methods": res, "tau_at_naive_fraction": tau}
        ctx.close()
        log(f"[deltar] {name}: " + ", ".join(f"{m} {r.get('n_prop_mean', r.get('n_prop'))}" for m, r in res.items()))
    # every tree method once on the 128x128 blob image (4-neighbours)
    img = synth.config2()
    ctx = gapd.Context(img, conn=4)
    big = {}
    for mname, kw in (("filling_rate", {"mode": gapd.MODE_TREE_FILL_FR}),
                      ("extrema", {"mode": gapd.MODE_TREE_FILL_EXTREMA}),
                      ("spiral", {"draws": synth.spiral_draws(0, img.size), "h": 0}),
                      ("spiral_repulsion3", {"draws": synth.spiral_draws(0, img.size), "h": 3})):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, _ = run(ctx, **kw)
        ms = (time.perf_counter() - t1) * 1e3
        big[mname] = {"n_prop": int(st.n_prop), "ms": round(ms, 1), "cache_hits": int(st.n_cache_hits)}
        log(f"[deltar] blob128 {mname}: n_prop {st.n_prop}, {ms:.0f} ms")
    wall = time.time() - t0
    return {"metric": "propagations to fill D, relative difference vs naive and spiral (Delta_r)",
            "value": out["bumps"]["methods"]["filling_rate"]["dr_naive_pct"], "unit": "% (bumps, filling rate)",
            "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(wall * 1e3, 1),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic", "config": {"workload": "deltar", "side": 25, "conn": conn,
                                            "weights": "f(p)+f(q)", "images": "synth.deltar_images(seed=7)"},
            "images": out, "blob128_all_methods": big}


def graph_line(args):
    """The general-graph path on a random geometric graph: filling rate vs naive."""
    import torch
    import synth
    from paper_2007_16076_amd import gapd
    n = 4096
    rp, ci, cw = synth.geometric_graph(np.random.default_rng(11), n)
    g = gapd.Graph(rp, ci, cw)
    res = {}
    for mode in (gapd.MODE_TREE_FILL_FR, gapd.MODE_NAIVE):
        out = torch.empty((n, n), dtype=torch.int32, device="cuda")
        sts, ms = [], []
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = g.all_pairs(mode, out=out, time_kernels=(mode != gapd.MODE_NAIVE))
            torch.cuda.synchronize()
            if i >= args.warmup:
                ms.append((time.perf_counter() - t0) * 1e3)
                sts.append(st)
        res[mode] = (sts, ms)
        log(f"[graph] mode={mode}: {np.mean(ms):.1f} ms, n_prop {sts[-1].n_prop}")
    fst, fms = res[gapd.MODE_TREE_FILL_FR]
    nst, nms = res[gapd.MODE_NAIVE]
    s0 = fst[-1]
    kern = float(np.mean([s.ms_kernel for s in nst]))
    roof = roofline_hbm(4.0 * n * n, kern)
    roof.update(kernel="k_graph_rows (one frontier Bellman-Ford propagation per workgroup, writes its row)",
                algorithmic_bytes_per_launch=4 * n * n, avg_launch_ms=round(kern, 4), traffic=None)
    return {"metric": METRIC, "value": n * n / (np.mean(fms) * 1e-3), "unit": "distance entries/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(float(np.mean(fms)), 3),
            "p50_ms": round(pct(fms, 50), 3), "p99_ms": round(pct(fms, 99), 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": "graph", "n": n, "edges_directed": int(rp[-1]),
                       "graph": "synth.geometric_graph(default_rng(11), 4096)", "mode": "tree_fill_filling_rate"},
            "n_prop": int(s0.n_prop), "n_prop_setup": int(s0.n_prop_setup),
            "propagation_saving_vs_naive": round(1.0 - (s0.n_prop + 2) / n, 4),
            "fr_loop_kernel_ms": {"select_propagate": round(s0.ms_step_kernels, 3),
                                  "fill": round(s0.ms_fill_kernels, 3)},
            "rounds_per_propagation": round(s0.rounds / max(s0.n_prop + 2, 1), 1),
            "naive": {"value": n * n / (np.mean(nms) * 1e-3), "ms_per_call": round(float(np.mean(nms)), 3),
                      "kernel_ms": round(kern, 3)},
            "roofline_naive": roof}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="blob128",
                    choices=["blob128", "uniform32", "voronoi192", "batched", "serve", "hbmcopy", "blob128c8",
                             "deltar", "graph"])
    ap.add_argument("--draw-seeds", type=int, default=10, help="deltar: draw sequences per spiral method")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of each oracle timing sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rate", type=float, default=30.0)
    ap.add_argument("--rates", default=None, metavar="R1,R2,...",
                    help="serve: sweep these arrival rates (req/s), one JSON line each")
    ap.add_argument("--requests", type=int, default=60)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--serve-mode", default="naive", choices=["naive", "tree_fill"])
    ap.add_argument("--fill-trace", default=None, metavar="CSV",
                    help="single-image workloads: one more filling-rate call with the per-step trace; "
                         "the summary joins the JSON line, the per-step table goes to CSV")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "only one GPU is supported: sharding the sources over several GPUs "
                                   "is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    import synth
    if args.workload == "blob128":
        img = synth.config2()
        line, _ = single_image_line(args, "blob128", img, 4,
                                    {"image": "128x128 sum of 20 Gaussian blobs + noise, seed 1",
                                     "weights": "f(p)+f(q)", "sha256": synth.sha256(img)})
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline_fr(img, 4, line["n_prop"], args.cpu_seconds)
            line["cpu_baseline_naive"] = cpu_baseline_naive(img, 4, args.cpu_seconds / 3)
    elif args.workload == "uniform32":
        img = synth.config1()
        line, _ = single_image_line(args, "uniform32", img, 4, {"image": "32x32 iid uniform [1,255], seed 0",
                                                                "weights": "f(p)+f(q)"}, fr=False)
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline_naive(img, 4, args.cpu_seconds)
    elif args.workload == "voronoi192":
        img = synth.config3()
        line, _ = single_image_line(args, "voronoi192", img, 4,
                                    {"image": "192x192x8 Voronoi, 50 regions, noise sigma 6, seed 2",
                                     "weights": "1 + L1 over 8 bands"})
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline_fr(img, 4, line["n_prop"], args.cpu_seconds)
    elif args.workload == "blob128c8":
        img = synth.config2()
        line, _ = single_image_line(args, "blob128c8", img, 8,
                                    {"image": "128x128 sum of 20 Gaussian blobs + noise, seed 1",
                                     "weights": "f(p)+f(q)", "sha256": synth.sha256(img)})
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline_fr(img, 8, line["n_prop"], args.cpu_seconds)
    elif args.workload == "deltar":
        line = deltar_line(args)
    elif args.workload == "graph":
        line = graph_line(args)
    elif args.workload == "batched":
        line = batched_line(args)
    elif args.workload == "hbmcopy":
        line = hbmcopy_line(args)
    elif args.rates:
        for r in [float(x) for x in args.rates.split(",")]:
            print(json.dumps(serve_line(args, r)), flush=True)
        return
    else:
        line = serve_line(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

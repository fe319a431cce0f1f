#!/usr/bin/env python3
"""Benchmark of the ENUFFT hot path on one MI355X.

Workload (default): 20,480 triangular cells of a 5x subdivided icosahedron in
local tangent-plane frames, lognormal point counts (median 2e4, sigma 1.2,
clipped 500..5e5; ~8e8 points), jittered-lattice positions with 30 % dropout,
200-sinusoid power-law terrain, uniform weights, radial Hann windows, 64 x 64
modes, sigma 2, FP32 with eps 1e-5, EMS keeping 95 % of the power.  Inputs are
synthetic and seeded (the paper's DEM data are not available).

A step is one pass of the whole hot path: batched type-1 (spread, FFT,
deconvolve, crop), EMS, and the type-2 adjoint giving d(sum retained power) /
d(h, x, y).  The JSON line reports NU points/s of type-1 + EMS (kernel time
from HIP events on the plan's stream), the fwd+bwd step time, the per-cell
launch loop on the same GPU, the spreading kernel against the HBM roofline and
the FP64 CPU oracle timed on a bounded sample of cells.  Parity of this exact
launch configuration against the oracle is checked by the GPU test suite
(full-size sampled cells), not here.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(batch, seconds, seed=1):
    """The FP64 oracle (type-1 direct sums + EMS) on a seeded sample of cells."""
    import oracle
    cnt = batch.counts()
    rng = np.random.default_rng(seed)
    order = [int(c) for c in rng.permutation(batch.n_cells) if cnt[c] > 0]
    # calibrate on one cell, then take cells until the predicted time fills the budget
    t0 = time.perf_counter()
    inp = oracle.batch_inputs(batch, [order[0]])
    f = oracle.type1(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"], inp["n_modes"],
                     kind=inp["kind"])
    oracle.ems_batched(f, oracle.EmsParams())
    rate = cnt[order[0]] / max(1e-6, time.perf_counter() - t0)
    cells, pts = [], 0
    for c in order[1:]:
        if (pts + cnt[c]) / rate > seconds:
            break
        cells.append(c)
        pts += int(cnt[c])
    if not cells:
        cells, pts = [order[1]], int(cnt[order[1]])
    inp = oracle.batch_inputs(batch, cells)
    t0 = time.perf_counter()
    f = oracle.type1(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"], inp["n_modes"],
                     kind=inp["kind"])
    oracle.ems_batched(f, oracle.EmsParams())
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": pts / dt, "unit": "NU points/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded cells, %d points, type-1 direct sums + EMS, %.1f s" % (len(cells), pts, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=None, help="first n cells only (debugging)")
    ap.add_argument("--no-percell", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--shuffled", action="store_true", help="random point order within each cell")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="after timing, run one plain device copy of this size (for profiler byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: every box here has a single MI355X and this build has no "
              "multi-GPU path (cells shard with no exchange; see the design notes). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, here)
    import paper_2606_21278_amd as enf
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    batch = synth.config3(device=dev, n_cells=args.cells, shuffled=args.shuffled)
    torch.cuda.synchronize()
    log("generated %s: %d cells, %d points in %.1f s" % (batch.name, batch.n_cells, batch.n_points,
                                                         time.perf_counter() - t0))
    gb = batch.to(device=dev, dtype=torch.float32)
    del batch.x, batch.y, batch.h, batch.w
    batch.x, batch.y, batch.h, batch.w = gb.x, gb.y, gb.h, gb.w
    plan = enf.Plan(gb.cell_offsets, gb.windows, n_modes=gb.n_modes, sigma=gb.sigma, eps=gb.eps, precision="f32")
    info = plan.info()
    log("plan", info)
    prm = enf.EmsParams()
    Q = batch.n_points
    M = gb.n_modes[0] * gb.n_modes[1]

    def step():
        f = plan.type1(gb.x, gb.y, gb.h, gb.w)
        keep, ks, st = plan.ems(f, prm)
        grads = plan.retained_power_adjoint(gb.x, gb.y, gb.h, gb.w, f, keep)
        return f, keep, ks, st, grads

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.get_timing()          # discard warm-up records
    plan.set_timing(True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    plan.set_timing(False)
    ms_step = e0.elapsed_time(e1) / args.steps
    tm = plan.get_timing()
    t1 = tm["type1_ms"] / max(1, tm["type1_launches"])
    tems = tm["ems_ms"] / max(1, tm["ems_launches"])
    tadj = tm["adjoint_ms"] / max(1, tm["adjoint_launches"])
    value = Q / ((t1 + tems) * 1e-3)
    log("per step: type1 %.3f ms, ems %.3f ms, adjoint %.3f ms, step %.3f ms" % (t1, tems, tadj, ms_step))

    if args.calibrate_copy > 0:
        n = args.calibrate_copy * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d MB read + %d MB written" % (args.calibrate_copy, args.calibrate_copy))
        del src, dst

    percell = None
    if not args.no_percell:
        plan.percell_loop(gb.x, gb.y, gb.h, gb.w, prm)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.percell_loop(gb.x, gb.y, gb.h, gb.w, prm)
        b.record(stream)
        torch.cuda.synchronize()
        pc_ms = a.elapsed_time(b)
        percell = {"value": Q / (pc_ms * 1e-3), "unit": "NU points/s", "ms": pc_ms,
                   "launches": 2 * batch.n_cells}
        log("per-cell loop %.1f ms" % pc_ms)

    fwd_bytes = 16.0 * Q + 8.0 * M * batch.n_cells        # read x, y, h, w; write f
    achieved = fwd_bytes / (t1 * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                "frac": achieved / 8000.0, "traffic": None, "kernel": "fwd_kernel (spread+FFT+deconv+crop)",
                "bytes_per_launch": fwd_bytes}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batch, args.cpu_seconds)
        log("cpu baseline", cpu)
    out = {
        "metric": "NU points/s batched type-1+EMS at rel-l2 5e-5 vs per-cell loop; fwd+bwd ms",
        "value": value, "unit": "NU points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded icosahedral-cell terrain)",
        "config": {"workload": "20,480 icosahedral triangles, ~8e8 points, 64x64 modes, sigma 2, eps 1e-5, "
                               "Hann window, EMS 95% power, fwd+bwd" if args.cells is None else
                               "first %d icosahedral triangles" % batch.n_cells,
                   "n_cells": batch.n_cells, "n_points": Q, "modes": list(gb.n_modes), "sigma": 2.0, "eps": 1e-5,
                   "kernel_width": info["kernel_width"], "grid": info["grid"]},
        "type1_ms": t1, "ems_ms": tems, "adjoint_ms": tadj, "fwd_bwd_ms": ms_step,
        "per_cell_loop": percell, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

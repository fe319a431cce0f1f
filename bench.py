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
launch loop on the same GPU, the forward kernel against the HBM roofline and
the FP64 CPU oracle timed on a bounded sample of cells (all host threads, and one).

Before anything is timed, the plan that is timed passes a parity gate: on a seeded
sample of cells (the two largest, the two smallest and four others) its FP32
coefficients must be within 5e-5 relative l2 of the FP64 oracle's per cell, its
EMS selection must equal the oracle's on the same coefficients, and its adjoint
must be within 5e-5 relative l2 of the oracle's; otherwise the script exits with
status 3 and times nothing.

Timing: the headline times type-1 + EMS as the captured HIP graph
(enufft_forward_graph), one replay per step, with HIP events on the plan's stream
around each replay; the adjoint follows each replay inside the timed steps.  A
second, separate set of eager steps records HIP events around every kernel
launch for the per-kernel breakdown and the forward kernel's roofline figure.

Profiles: ``--summarize DIR`` turns rocprofv3 output collected from this script
(kernel-trace stats CSV and FETCH_SIZE / WRITE_SIZE counter CSVs) into the
text summaries and the traffic record kept under profiles/.
"""
import argparse
import csv
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "c3_kernels_hbm_traffic.json")
# the main kernels of a step and the sources whose text fixes each one's code
# (a kernel's counter record is void once they change)
KERNEL_SOURCES = {
    "fwd_kernel": ["paper_2606_21278_amd/csrc/fwd.hip", "paper_2606_21278_amd/csrc/device_common.h",
                   "paper_2606_21278_amd/csrc/launch.h"],
    "ems_kernel": ["paper_2606_21278_amd/csrc/ems.hip", "paper_2606_21278_amd/csrc/device_common.h"],
    "adj_kernel": ["paper_2606_21278_amd/csrc/adj.hip", "paper_2606_21278_amd/csrc/device_common.h",
                   "paper_2606_21278_amd/csrc/launch.h"],
    "adj1_kernel": ["paper_2606_21278_amd/csrc/adj.hip", "paper_2606_21278_amd/csrc/device_common.h",
                    "paper_2606_21278_amd/csrc/launch.h"],
}
FWD_KERNEL = "fwd_kernel"
COPY_KERNEL = "bitwise_not"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(kernel):
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def fwd_source_hash():
    return source_hash(FWD_KERNEL)


def measured_traffic(kernel=FWD_KERNEL):
    """HBM bytes per launch of a kernel from the committed counter record, if it was
    taken with the kernel's current source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("source_hash") != source_hash(kernel):
        return None
    return k.get("bytes_per_launch")


def _omp_threads(n):
    """Set the OpenMP thread count of the oracle's runtime (None: leave it)."""
    import ctypes
    import ctypes.util
    if n is None:
        return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    lib = ctypes.CDLL(ctypes.util.find_library("gomp") or "libgomp.so.1")
    lib.omp_set_num_threads(int(n))
    return int(n)


def cpu_baseline(batch, seconds, seed=1, threads=None):
    """The FP64 oracle (type-1 direct sums + EMS) on a seeded sample of cells."""
    import oracle
    oracle.type1([0, 0], np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0), [[0, 0, 1]], (2, 2))  # load
    threads = _omp_threads(threads)
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
    return {"value": pts / dt, "unit": "NU points/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded cells, %d points, type-1 direct sums + EMS, %.1f s" % (len(cells), pts, dt)}


def cpu_baseline_points(batch, seconds, seed=1):
    """The FP64 oracle's type-1 direct sums + EMS on a seeded sample of one cell's
    points (all modes), scaled to points per second."""
    import oracle
    rng = np.random.default_rng(seed)
    N1, N2 = batch.n_modes
    win = batch.windows[:1]

    def run(n):
        idx = np.sort(rng.choice(batch.n_points, size=n, replace=False))
        it = __import__("torch").as_tensor(idx, device=batch.x.device)
        g = lambda t: t[it].cpu().double().numpy()
        x, y, h, w = g(batch.x), g(batch.y), g(batch.h), g(batch.w)
        off = np.array([0, n], dtype=np.int64)
        t0 = time.perf_counter()
        f = oracle.type1(off, x, y, h, w, win, (N1, N2), kind=1)
        oracle.ems_batched(f, oracle.EmsParams())
        return time.perf_counter() - t0

    n = 2000
    dt = run(n)
    n = int(min(batch.n_points, max(n, n * seconds / max(dt, 1e-6))))
    dt = run(n)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n / dt, "unit": "NU points/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded points of the cell, type-1 direct sums over all %dx%d modes + EMS, %.1f s"
                      % (n, N1, N2, dt)}


def bench_c4(args, torch, enf, synth, dev):
    """The single high-resolution cell: 1e8 clustered points, 512 x 512 modes on a
    1024^2 grid (tile sort, tiled spreading into HBM, row/column FFT passes, EMS over
    131,583 units with the device sort, tiled adjoint)."""
    t0 = time.perf_counter()
    b = synth.config4(device=dev, Q=args.points, precision=args.precision,
                      progress=lambda s: log("generating: %s (%.0f s)" % (s, time.perf_counter() - t0)))
    torch.cuda.synchronize()
    log("generated %s in %.1f s" % (b.name, time.perf_counter() - t0))
    plan = enf.Plan(b.cell_offsets, b.windows, n_modes=b.n_modes, sigma=b.sigma, eps=b.eps,
                    precision=args.precision)
    info = plan.info()
    log("plan", info)
    prm = enf.EmsParams()
    Q = b.n_points
    N1, N2 = b.n_modes
    sort_rec = None
    if not args.no_sort:
        # sorted once by tile: every later call's counting pass finds the order and skips
        # its scatter
        plan.sort_points(b.x, b.y, b.h, b.w)
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(torch.cuda.current_stream())
        xs, ys, hs, ws, _ = plan.sort_points(b.x, b.y, b.h, b.w)
        s1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        sort_rec = {"ms": s0.elapsed_time(s1), "note": "tile sort of the cell (enufft_sort_points), once, before "
                                                        "timing; the timed calls run on the sorted copies"}
        b.x, b.y, b.h, b.w = xs, ys, hs, ws
        if not args.no_bind:
            # the sorted coordinates bound once: the timed calls sort nothing
            s0.record(torch.cuda.current_stream())
            plan.bind_points(b.x, b.y)
            s1.record(torch.cuda.current_stream())
            torch.cuda.synchronize()
            sort_rec["bind_ms"] = s0.elapsed_time(s1)
            sort_rec["note"] += "; the sorted x and y bound to the plan (enufft_bind_points), once"
        log("sort", sort_rec)

    def step():
        f = plan.type1(b.x, b.y, b.h, b.w)
        keep, ks, st = plan.ems(f, prm)
        grads = plan.retained_power_adjoint(b.x, b.y, b.h, b.w, f, keep)
        return f, keep, ks, st, grads

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warm-up step %d done" % (i + 1))
    plan.get_timing()
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
    log("per step: type1 %.3f ms, ems %.3f ms, adjoint %.3f ms, step %.3f ms" % (t1, tems, tadj, ms_step))
    el = 8 if args.precision == "f64" else 4
    # algorithmic bytes of the type-1 pass: read x, y, h, w; write f
    t1_bytes = 4.0 * el * Q + 2.0 * el * N1 * N2
    achieved = t1_bytes / (t1 * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                "traffic": None, "kernel": "type-1 pass (tile sort + tiled spreading + row/column FFT passes)",
                "bytes_per_launch": t1_bytes, "avg_launch_ms": t1}
    cpu = None if args.no_cpu_baseline else cpu_baseline_points(b, args.cpu_seconds)
    if cpu:
        log("cpu baseline", cpu)
    out = {
        "metric": "NU points/s batched type-1+EMS at rel-l2 5e-5 vs per-cell loop; fwd+bwd ms",
        "value": Q / ((t1 + tems) * 1e-3), "unit": "NU points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.precision, "data": "synthetic (seeded clustered hexagon terrain)",
        "config": {"workload": "one hexagon, %d clustered points, %dx%d modes, sigma 2, eps %g, Hann window, "
                               "EMS 95%% power, fwd+bwd" % (Q, N1, N2, b.eps),
                   "n_cells": 1, "n_points": Q, "modes": [N1, N2], "sigma": 2.0, "eps": b.eps,
                   "kernel_width": info["kernel_width"], "grid": info["grid"]},
        "type1_ms": t1, "ems_ms": tems, "adjoint_ms": tadj, "fwd_bwd_ms": ms_step,
        "per_cell_loop": None, "roofline": roofline, "cpu_baseline": cpu, "sort": sort_rec,
    }
    print(json.dumps(out), flush=True)


def make_plan(enf, gb, workload="c3", shuffled=False, autotune=True, sorted_points=False):
    """The plan this script times.  The autotuner's trial points follow the order the
    type-1 spreads: the icosahedral cells store their samples in raster order, the
    hexagons (and the shuffled variant) in no spatial order unless they are sorted
    by fine cell first."""
    tune = ("unordered" if (workload == "c1" or shuffled) and not sorted_points else "raster") if autotune else False
    return enf.Plan(gb.cell_offsets, gb.windows, n_modes=gb.n_modes, sigma=gb.sigma, eps=gb.eps, precision="f32",
                    autotune=tune)


def reconstruction_figures(plan, gb, f, keep, torch, steps):
    """The Section 3.2 diagnostics over the whole batch: the truncated series over the
    kept modes at every sample, eps_rel and the Parseval ratio per cell, from the
    coefficients normalised by the cell areas (the paper's hat h).  Timed with HIP
    events on the plan's stream (one enufft_reconstruct per step)."""
    area = torch.as_tensor(gb.areas, dtype=torch.float64, device=gb.x.device)
    coef = (f * (1.0 / area).to(torch.float32)[:, None, None]).contiguous()
    # the same with the box area (2 pi)^2 in place of the cell's: the series then
    # represents the windowed field itself on the periodic box
    box = (2 * np.pi) ** 2
    _, dgb = plan.reconstruct(gb.x, gb.y, gb.h, gb.w, (f * (1.0 / box)).contiguous(), keep,
                              torch.full_like(area, box), need_h_rec=False)
    plan.reconstruct(gb.x, gb.y, gb.h, gb.w, coef, keep, area, need_h_rec=False)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    dg = None
    for e0, e1 in e:
        e0.record(s)
        _, dg = plan.reconstruct(gb.x, gb.y, gb.h, gb.w, coef, keep, area, need_h_rec=False)
        e1.record(s)
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in e]))
    d = dg.cpu().numpy()
    db = dgb.cpu().numpy()
    live = d[:, 0] > 0
    return {"ms": ms, "points_per_s": float(gb.n_points / (ms * 1e-3)),
            "box_normalised": {"eps_rel_median": float(np.median(db[live, 6])),
                               "parseval_ratio_median": float(np.median(db[live, 7])),
                               "parseval_ratio_kept_median": float(np.median(db[live, 5] / db[live, 3]))},
            "eps_rel_median": float(np.median(d[live, 6])), "eps_rel_p90": float(np.percentile(d[live, 6], 90)),
            "parseval_ratio_median": float(np.median(d[live, 7])),
            "parseval_ratio_kept_median": float(np.median(d[live, 5] / d[live, 3])),
            "note": "eq. alps_relative_rmse and eq. spectral_variance per cell, kept modes, target W h; "
                    "|D| = cell area as printed (the series then carries |B|/|D| on the square box B), "
                    "and |D| = |B| = (2 pi)^2"}


def flow_selection_figures(plan, gb, f, prm, torch, steps, n_t=8, seed=5):
    """EMS re-selected over n_t timesteps on the fixed coefficients, with a seeded
    flow record per step and cell (wind ~ N(0, 8 m/s) per component, N in
    [0.01, 0.025] 1/s, fc 1e-4 1/s, cells of 80 km): one enufft_ems_flow launch for
    all steps, timed with HIP events on the plan's stream."""
    rng = np.random.default_rng(seed)
    fl = np.zeros((n_t, gb.n_cells, 6))
    fl[..., 0:2] = rng.normal(scale=8.0, size=(n_t, gb.n_cells, 2))
    fl[..., 2] = rng.uniform(0.01, 0.025, size=(n_t, gb.n_cells))
    fl[..., 3] = 1e-4
    fl[..., 4] = 1.0
    fl[..., 5] = 2 * np.pi / 80000.0
    flow = torch.as_tensor(fl, device=gb.x.device)
    plan.ems_flow(f, flow, prm)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    ks = None
    for e0, e1 in e:
        e0.record(s)
        _, ks, _ = plan.ems_flow(f, flow, prm)
        e1.record(s)
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in e]))
    k = ks.cpu().numpy()
    return {"timesteps": n_t, "ms": ms, "ms_per_timestep": ms / n_t,
            "cell_selections_per_s": float(n_t * gb.n_cells / (ms * 1e-3)),
            "k_star_median": float(np.median(k)), "k_star_changed_between_steps": float(np.mean(k[1:] != k[:-1]))}


def geometry_figures(plan, gb, torch, synth, steps):
    """enufft_cell_geometry over the whole batch (the icosahedral triangles the cells
    lie on): edge frame, triangle mask, deplaning, with raster-Voronoi weights (N_g =
    64) and with uniform weights; HIP events on the plan's stream.  Algorithmic bytes
    per point: x, y, h read (3 reals) and xb, yb, hb, wb and the mask byte written."""
    tri = synth.local_triangles(5)[:gb.n_cells].reshape(-1, 6)
    out = {}
    el = gb.x.element_size()
    for wk in ("voronoi", "uniform"):
        kw = dict(frame="edge", mask="triangle", weights=wk, raster=64, eta=1.0, deplane=True, need_info=False)
        plan.cell_geometry(tri, gb.x, gb.y, gb.h, **kw)
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for e0, e1 in e:
            e0.record(s)
            g = plan.cell_geometry(tri, gb.x, gb.y, gb.h, **kw)
            e1.record(s)
            del g
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in e]))
        byts = (7 * el + 1) * gb.n_points
        out[wk] = {"ms": ms, "points_per_s": float(gb.n_points / (ms * 1e-3)),
                   "achieved_GBps": byts / (ms * 1e-3) / 1e9, "hbm_frac": byts / (ms * 1e-3) / 8e12}
    torch.cuda.empty_cache()
    out["note"] = "edge frame, triangle mask, deplaning; Voronoi N_g = 64 raster"
    return out


def gate_cells(counts, seed=7, n_random=4):
    """The parity gate's cells: the two largest, the two smallest non-empty and
    n_random seeded others."""
    order = [int(c) for c in np.argsort(counts, kind="stable") if counts[c] > 0]
    rng = np.random.default_rng(seed)
    rest = [c for c in order[2:-2]]
    pick = [int(c) for c in rng.choice(rest, size=min(n_random, len(rest)), replace=False)] if rest else []
    return sorted(set(order[-2:] + order[:2] + pick))


def parity_gate(plan, gb, prm, torch, tol=5e-5):
    """Run the timed plan once (type-1, EMS, retained-power adjoint) and check a
    seeded sample of cells against the FP64 oracle: per-cell rel-l2 of the
    coefficients, the EMS selection on the same coefficients (exact), and the
    adjoint's rel-l2 per gradient component over the sample's points."""
    import oracle
    cells = gate_cells(gb.counts())
    f = plan.type1(gb.x, gb.y, gb.h, gb.w)
    keep, ks, st = plan.ems(f, prm)
    gh, gx, gy = plan.retained_power_adjoint(gb.x, gb.y, gb.h, gb.w, f, keep)
    torch.cuda.synchronize()
    sub = gb.subset(cells).to(device="cpu")
    inp = oracle.batch_inputs(sub)
    ref = oracle.type1(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"], inp["n_modes"],
                       kind=inp["kind"])
    fg = f[cells].cpu().numpy().astype(np.complex128)
    rel = [float(np.linalg.norm(fg[i] - ref[i]) / max(np.linalg.norm(ref[i]), 1e-300)) for i in range(len(cells))]
    oprm = oracle.EmsParams(**{k: getattr(prm, k) for k in oracle.EmsParams.__dataclass_fields__})
    ok_keep, ok_ks, _ = oracle.ems_batched(fg, oprm)
    ems_ok = bool(np.array_equal(ok_ks, ks[cells].cpu().numpy()) and
                  np.array_equal(ok_keep, keep[cells].cpu().numpy()))
    g = 2.0 * fg * ok_keep
    rh, rx, ry = oracle.type1_vjp(inp["offsets"], inp["x"], inp["y"], inp["h"], inp["w"], inp["windows"],
                                  inp["n_modes"], g, kind=inp["kind"])
    idx = np.concatenate([np.arange(gb.cell_offsets[c], gb.cell_offsets[c + 1]) for c in cells])
    it = torch.as_tensor(idx, device=gb.x.device)
    grel = {}
    for name, got, want in (("h", gh, rh), ("x", gx, rx), ("y", gy, ry)):
        a = got[it].cpu().double().numpy()
        grel[name] = float(np.linalg.norm(a - want) / max(np.linalg.norm(want), 1e-300))
    ok = max(rel) <= tol and ems_ok and max(grel.values()) <= tol
    return {"pass": bool(ok), "cells": cells, "points": int(len(idx)), "coef_rel_l2_max": max(rel),
            "ems_identical": ems_ok, "grad_rel_l2": grel, "tol": tol}


def bench_kernel_study(args, torch, enf, synth, dev):
    """The spreading kernels compared as in the kernel study of Section 2.1.2: three
    seeded power-law terrains of 2,000 samples on the square box, modes |m|, |n| <= 20,
    kernel width 2a = 8, oversampling 1.25, 1.5 and 2; per coefficient the error
    e = log10 |f_NUFFT - f_DFT| against the oracle's direct sums (FP64 on both sides,
    coefficients normalised by the box area).  Then the FP32 type-1 launch on the
    20,480-cell batch with each kernel (HIP events), for throughput."""
    import oracle
    t0 = time.perf_counter()
    terr = [synth.square_terrain(device=dev, seed=s) for s in range(3)]
    refs = [oracle.type1(b.cell_offsets, b.x.cpu().numpy(), b.y.cpu().numpy(), b.h.cpu().numpy(),
                         b.w.cpu().numpy(), b.windows, b.n_modes, scale=1.0 / b.areas[0], kind=0) for b in terr]
    study = []
    for kern in ("es", "kb_mirt", "kb_fessler"):
        for sigma in (1.25, 1.5, 2.0):
            errs, rels, info = [], [], None
            for b, ref in zip(terr, refs):
                plan = enf.Plan(b.cell_offsets, None, n_modes=b.n_modes, sigma=sigma, eps=1e-3, precision="f64",
                                window="none", scale=1.0 / b.areas[0], kernel=kern, kernel_width=8)
                info = plan.info()
                f = plan.type1(b.x, b.y, b.h, b.w).cpu().numpy()
                d = np.abs(f - ref).ravel()
                errs.append(np.log10(np.maximum(d, 1e-300)))
                rels.append(float(np.linalg.norm(f - ref) / np.linalg.norm(ref)))
            e = np.concatenate(errs)
            study.append({"kernel": kern, "sigma": sigma, "grid": info["grid"], "width": info["kernel_width"],
                          "shape": info["beta"], "log10_err_median": float(np.median(e)),
                          "log10_err_p10": float(np.percentile(e, 10)), "log10_err_p90": float(np.percentile(e, 90)),
                          "rel_l2_max": max(rels)})
            log(study[-1])
    # throughput on the 20,480-cell batch (FP32, eps 1e-5, default launch shape)
    batch = synth.config3(device=dev)
    gb = batch.to(device=dev, dtype=torch.float32)
    speed = {}
    for kern in ("es", "kb_mirt"):
        plan = enf.Plan(gb.cell_offsets, gb.windows, n_modes=gb.n_modes, sigma=gb.sigma, eps=gb.eps,
                        precision="f32", kernel=kern)
        f = plan.type1(gb.x, gb.y, gb.h, gb.w)
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for e0, e1 in ev:
            e0.record(s)
            plan.type1(gb.x, gb.y, gb.h, gb.w, out=f)
            e1.record(s)
        torch.cuda.synchronize()
        inf = plan.info()
        speed[kern] = {"type1_ms": float(np.median([a.elapsed_time(b2) for a, b2 in ev])),
                       "width": inf["kernel_width"], "poly_err": inf["kernel_poly_err"]}
        log(kern, speed[kern])
    print(json.dumps({"study": "spreading kernels (Section 2.1.2)", "accuracy": study, "c3_type1": speed,
                      "seconds": time.perf_counter() - t0}), flush=True)


# ------------------------------------------------------------------ profile summaries

def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _short(name):
    name = name.split("(")[0]
    return name if len(name) < 90 else name[:87] + "..."


def summarize(d, command_trace, command_fetch, command_write, copy_mb):
    """Write profiles/ summaries from rocprofv3 CSVs in directory d:
    *kernel_stats.csv (kernel trace), fetch*counter_collection.csv, write*counter_collection.csv.
    Covers the forward, EMS and adjoint kernels of the benchmark's step."""
    out_dir = os.path.join(HERE, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    stats = sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True))
    lines = ["# Kernels of the C3 step (type-1, EMS, adjoint): kernel-trace statistics", "",
             "Command (repo root, one MI355X):", "", "    " + command_trace, "",
             "Source hashes: " + ", ".join("%s `%s`" % (k, source_hash(k)) for k in KERNEL_SOURCES), "",
             "| kernel | calls | total ms | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    avg_us = {}
    if stats:
        rows = _rows(stats[0])
        # the largest entries (the synthetic data generation's among them), then the
        # step's own kernels wherever they rank
        ours = [r for r in rows if any(("::" + k + "<") in r["Name"] for k in KERNEL_SOURCES)]
        for r in rows[:10] + [r for r in ours if r not in rows[:10]]:
            avg = float(r["AverageNs"]) / 1e3
            lines.append("| %s | %s | %.3f | %.2f | %.2f | %.2f | %.2f |" % (
                _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6, avg,
                float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
        for r in ours:
            for k in KERNEL_SOURCES:
                if ("::" + k + "<") in r["Name"] and k not in avg_us:
                    avg_us[k] = float(r["AverageNs"]) / 1e3
    with open(os.path.join(out_dir, "c3_kernels_kernel_trace.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    def per_dispatch(pattern, counter):
        files = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
        vals = {}
        for fpath in files:
            for r in _rows(fpath):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"]
                key = COPY_KERNEL if COPY_KERNEL in name else next(
                    (k for k in KERNEL_SOURCES if ("::" + k + "<") in name), None)
                if key:
                    vals.setdefault(key, []).append(float(r["Counter_Value"]))
        return vals

    fetch = per_dispatch("fetch*counter_collection.csv", "FETCH_SIZE")
    write = per_dispatch("write*counter_collection.csv", "WRITE_SIZE")
    copy_bytes = copy_mb * 1024.0 * 1024.0
    res = {"command_fetch": command_fetch, "command_write": command_write, "copy_mb": copy_mb, "kernels": {}}
    if fetch.get(COPY_KERNEL) and write.get(COPY_KERNEL):
        # counters are KiB per dispatch; scale by what they read for a copy of known size
        sf = copy_bytes / (max(fetch[COPY_KERNEL]) * 1024.0)
        sw = copy_bytes / (max(write[COPY_KERNEL]) * 1024.0)
        res.update({"fetch_scale": sf, "write_scale": sw})
        for k in KERNEL_SOURCES:
            if fetch.get(k) and write.get(k):
                fb = float(np.median(fetch[k])) * 1024.0 * sf
                wb = float(np.median(write[k])) * 1024.0 * sw
                res["kernels"][k] = {"source_hash": source_hash(k), "fetch_bytes": fb, "write_bytes": wb,
                                     "bytes_per_launch": fb + wb, "dispatches": len(fetch[k]),
                                     "trace_avg_us": avg_us.get(k)}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(res, fh, indent=1)
    lines = ["# Kernels of the C3 step: HBM traffic counters", "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two separate rocprofv3 passes:", "",
             "    " + command_fetch, "    " + command_write, "",
             "Each counter is scaled by what it reads for a plain streaming kernel (bitwise_not of %d MiB "
             "int32, read once and written once) in the same run: FETCH x %.4g, WRITE x %.4g."
             % (copy_mb, res.get("fetch_scale", float("nan")), res.get("write_scale", float("nan"))), "",
             "| kernel | fetch GB | write GB | total GB per launch | trace average us | source hash |",
             "|---|---|---|---|---|---|"]
    for k, v in res["kernels"].items():
        lines.append("| %s | %.3f | %.3f | %.3f | %s | `%s` |" % (
            k, v["fetch_bytes"] / 1e9, v["write_bytes"] / 1e9, v["bytes_per_launch"] / 1e9,
            "%.1f" % v["trace_avg_us"] if v["trace_avg_us"] else "-", v["source_hash"]))
    with open(os.path.join(out_dir, "c3_kernels_hbm_traffic.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps(res))


# ------------------------------------------------------------------ benchmark

def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=None, help="first n cells only (debugging)")
    ap.add_argument("--no-percell", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the reconstruction, flow-EMS and geometry figures (profiling runs: every "
                         "launch of the step's kernels is then one of the timed step's)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--shuffled", action="store_true", help="random point order within each cell")
    ap.add_argument("--no-sort", action="store_true",
                    help="unordered workloads: spread in the given order instead of sorting the points first")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="plan with the default launch shape instead of the autotuner's choice")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="after timing, run one plain device copy of this size (for profiler byte counters)")
    ap.add_argument("--summarize", metavar="DIR", help="write profiles/ summaries from rocprofv3 CSVs in DIR")
    ap.add_argument("--cmd-trace", default="")
    ap.add_argument("--cmd-fetch", default="")
    ap.add_argument("--cmd-write", default="")
    ap.add_argument("--workload", choices=["c1", "c3", "c4", "kernel-study"], default="c3",
                    help="c3: the 20,480-cell batch (default); c1: the 256-hexagon batch; "
                         "c4: the single high-resolution cell")
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32", help="c4 only")
    ap.add_argument("--points", type=int, default=100_000_000, help="c4 only: points in the cell")
    ap.add_argument("--no-bind", action="store_true",
                    help="c4 only: do not bind the sorted coordinates (every call runs the tile count)")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize, args.cmd_trace, args.cmd_fetch, args.cmd_write, args.calibrate_copy or 1024)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (cells are independent and "
              "would shard across GPUs with no exchange). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    sys.path.insert(0, HERE)
    import paper_2606_21278_amd as enf
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "c4":
        bench_c4(args, torch, enf, synth, dev)
        return
    if args.workload == "kernel-study":
        bench_kernel_study(args, torch, enf, synth, dev)
        return
    t0 = time.perf_counter()
    c1 = args.workload == "c1"
    if c1:
        batch = synth.config1(device=dev, **({"n_cells": args.cells} if args.cells else {}))
    else:
        batch = synth.config3(device=dev, n_cells=args.cells, shuffled=args.shuffled,
                              progress=lambda s: log("generating: %s (%.0f s)" % (s, time.perf_counter() - t0)))
    torch.cuda.synchronize()
    log("generated %s: %d cells, %d points in %.1f s" % (batch.name, batch.n_cells, batch.n_points,
                                                         time.perf_counter() - t0))
    gb = batch.to(device=dev, dtype=torch.float32)
    del batch.x, batch.y, batch.h, batch.w
    batch.x, batch.y, batch.h, batch.w = gb.x, gb.y, gb.h, gb.w
    # unordered samples (the hexagons, the shuffled variant) are sorted once by fine cell
    # (enufft_sort_points) and the timed calls work on the sorted copies
    sort = (c1 or args.shuffled) and not args.no_sort
    plan = make_plan(enf, gb, "c1" if c1 else "c3", args.shuffled, args.autotune, sort)
    info = plan.info()
    log("plan", info)
    sort_rec = None
    if sort:
        plan.sort_points(gb.x, gb.y, gb.h, gb.w)
        torch.cuda.synchronize()
        s_ = torch.cuda.current_stream()
        b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b0.record(s_)
        xs, ys, hs, ws, _ = plan.sort_points(gb.x, gb.y, gb.h, gb.w)
        b1.record(s_)
        torch.cuda.synchronize()
        bms = b0.elapsed_time(b1)
        # algorithmic bytes of the counting sort: x, y read twice (count, rank), h, w
        # read once; the permutation and the four sorted arrays written (the gather
        # pass also reads the permutation back and x, y a third time)
        bb = 44.0 * batch.n_points
        sort_rec = {"ms": bms, "bytes": bb, "achieved_GBps": bb / (bms * 1e-3) / 1e9,
                    "note": "per-cell counting sort by fine cell (enufft_sort_points), once, before timing; "
                            "the timed steps work on the sorted copies"}
        log("sort", sort_rec)
        gb.x, gb.y, gb.h, gb.w = xs, ys, hs, ws
        batch.x, batch.y, batch.h, batch.w = xs, ys, hs, ws
    prm = enf.EmsParams()
    Q = batch.n_points
    M = gb.n_modes[0] * gb.n_modes[1]

    gate = parity_gate(plan, gb, prm, torch)
    log("parity gate", gate)
    if not gate["pass"]:
        log("parity gate FAILED: nothing is timed")
        sys.exit(3)

    # headline: type-1 + EMS as one captured graph per step, then the adjoint
    out_t = (plan.empty_modes(), torch.empty((gb.n_cells, gb.n_modes[1], gb.n_modes[0]), dtype=torch.uint8,
                                             device=dev),
             torch.empty(gb.n_cells, dtype=torch.int32, device=dev),
             torch.empty((gb.n_cells, 8), dtype=torch.float64, device=dev))

    def step_graph():
        plan.forward_graph(gb.x, gb.y, gb.h, gb.w, prm, out=out_t)

    def step_adjoint():
        return plan.retained_power_adjoint(gb.x, gb.y, gb.h, gb.w, out_t[0], out_t[1])

    for i in range(args.warmup):
        step_graph()
        step_adjoint()
        torch.cuda.synchronize()
        log("warm-up step %d done" % (i + 1))
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step_graph()
        ev[i][1].record(stream)
        step_adjoint()
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    ms_step = ev[0][0].elapsed_time(ev[-1][2]) / args.steps
    graph_ms = np.array([e[0].elapsed_time(e[1]) for e in ev])
    adj_step_ms = np.array([e[1].elapsed_time(e[2]) for e in ev])
    t_fwd = float(np.median(graph_ms))
    value = Q / (t_fwd * 1e-3)
    log("graph type-1 + EMS: median %.3f ms (min %.3f, max %.3f); adjoint %.3f ms; step %.3f ms"
        % (t_fwd, graph_ms.min(), graph_ms.max(), float(np.median(adj_step_ms)), ms_step))

    # breakdown: eager launches with HIP events around every kernel launch
    plan.get_timing()
    plan.set_timing(True)
    for _ in range(args.steps):
        f = plan.type1(gb.x, gb.y, gb.h, gb.w)
        keep, ks, st = plan.ems(f, prm)
        plan.retained_power_adjoint(gb.x, gb.y, gb.h, gb.w, f, keep)
    torch.cuda.synchronize()
    plan.set_timing(False)
    tm = plan.get_timing()
    t1 = tm["type1_ms"] / max(1, tm["type1_launches"])
    tems = tm["ems_ms"] / max(1, tm["ems_launches"])
    tadj = tm["adjoint_ms"] / max(1, tm["adjoint_launches"])
    log("eager per launch: type1 %.3f ms, ems %.3f ms, adjoint %.3f ms" % (t1, tems, tadj))
    recon = flow_sel = geo = None
    if not args.no_extras:
        recon = reconstruction_figures(plan, gb, f, keep, torch, args.steps)
        log("reconstruction", recon)
        flow_sel = flow_selection_figures(plan, gb, f, prm, torch, args.steps)
        log("flow-dependent EMS", flow_sel)
    if not c1 and not args.no_extras:
        geo = geometry_figures(plan, gb, torch, synth, args.steps)
        log("mesh geometry", geo)

    if args.calibrate_copy > 0:
        # one streaming kernel of known traffic whose name no other kernel of this run shares
        n = args.calibrate_copy * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        log("copy calibration: %d MiB read + %d MiB written" % (args.calibrate_copy, args.calibrate_copy))
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
                   "launches": 2 * batch.n_cells, "batched_speedup": pc_ms / t_fwd}
        log("per-cell loop %.1f ms" % pc_ms)

    # algorithmic bytes of one forward launch: read x, y, h, w (16 B per point), write f (8 B per mode)
    fwd_bytes = 16.0 * Q + 8.0 * M * batch.n_cells
    achieved = fwd_bytes / (t1 * 1e-3) / 1e9
    traffic = measured_traffic(FWD_KERNEL) if (args.cells is None and not c1) else None   # counters taken on C3
    roofline = {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                "frac": achieved / 8000.0, "traffic": traffic, "kernel": "fwd_kernel (spread+FFT+deconv+crop)",
                "bytes_per_launch": fwd_bytes, "avg_launch_ms": t1}
    # the other two kernels of the step against the same roofline (algorithmic bytes per
    # launch: EMS reads f and writes the keep bytes; the adjoint reads x, y, h, w, f and keep
    # and writes three gradients)
    ems_bytes = 9.0 * M * batch.n_cells
    adj_bytes = 28.0 * Q + 9.0 * M * batch.n_cells
    others = {}
    adj_name = "adj1_kernel" if info.get("adj_kernel_width") else "adj_kernel"
    for k, byts, ms in (("ems_kernel", ems_bytes, tems), (adj_name, adj_bytes, tadj)):
        ach = byts / (ms * 1e-3) / 1e9
        others[k] = {"bound": "hbm", "achieved": ach, "peak": 8000.0, "unit": "GB/s", "frac": ach / 8000.0,
                     "traffic": measured_traffic(k) if (args.cells is None and not c1) else None,
                     "bytes_per_launch": byts, "avg_launch_ms": ms}
    cpu = cpu1 = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batch, args.cpu_seconds)
        log("cpu baseline", cpu)
        cpu1 = cpu_baseline(batch, args.cpu_seconds / 2, seed=2, threads=1)
        log("cpu baseline, one thread", cpu1)
    out = {
        "metric": "NU points/s batched type-1+EMS at rel-l2 5e-5 vs per-cell loop; fwd+bwd ms",
        "value": value, "unit": "NU points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded %s terrain)" % ("hexagon" if c1 else "icosahedral-cell"),
        "config": {"workload": ("256 hexagons, lognormal counts (median 2e4, sigma 1.0), 64x64 modes, sigma 2, "
                                "eps 1e-5, Hann window, EMS 95% power, fwd+bwd" if c1 else
                                "20,480 icosahedral triangles, ~8e8 points, 64x64 modes, sigma 2, eps 1e-5, "
                                "Hann window, EMS 95% power, fwd+bwd") if args.cells is None else
                               "first %d %s" % (batch.n_cells, "hexagons" if c1 else "icosahedral triangles"),
                   "n_cells": batch.n_cells, "n_points": Q, "modes": list(gb.n_modes), "sigma": 2.0, "eps": 1e-5,
                   "kernel_width": info["kernel_width"], "grid": info["grid"],
                   "fwd_threads": info["fwd_threads"], "autotuned": bool(info["tuned"])},
        "type1_ms": t1, "ems_ms": tems, "adjoint_ms": tadj, "fwd_bwd_ms": ms_step,
        "graph_type1_ems_ms": {"median": t_fwd, "mean": float(graph_ms.mean()), "min": float(graph_ms.min()),
                               "max": float(graph_ms.max())},
        "adjoint_in_step_ms": float(np.median(adj_step_ms)),
        "reconstruction": recon, "flow_ems": flow_sel, "mesh_geometry": geo, "sort": sort_rec,
        "parity_gate": gate, "plan": {k: info[k] for k in ("fwd_threads", "fwd_chunk_min", "fwd_items_per_slot",
                                                           "adj_items_per_slot", "adj_band_mult", "fwd_acc", "n_items_fwd",
                                                           "n_split_cells", "n_items_adj", "tuned")},
        "per_cell_loop": percell, "roofline": roofline, "roofline_other_kernels": others, "cpu_baseline": cpu,
        "cpu_baseline_1core": cpu1,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

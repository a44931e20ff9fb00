"""Benchmark of the FP64 sweep on the 4096^2 disc (one MI355X).

A step is one full sweep of the grid: slopes, characteristic limiting and
tracing, HLL fluxes, unsplit update, external-potential kick and the fused
CFL reduction that sets the next timestep on the device.  The timed region
replays the captured graph of K steps from the initial state, already
resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 50] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_CELL_F64 = 96     # 6 conserved planes read + 6 written, 8 B each
BYTES_PER_CELL_F32 = 48
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def time_graph(g, U0, steps):
    import torch
    g.U.copy_(U0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    dts = g.run_cfl(steps, 0.8)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, dts


def time_kernel(g, U0, steps, dt):
    """Average duration of the sweep kernel alone: back-to-back csh_step
    launches on the handle's stream, bracketed by HIP events."""
    import torch
    a, b = U0.clone(), torch.empty_like(U0)
    g.step(dt, a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        g.step(dt, a, b) if k % 2 == 0 else g.step(dt, b, a)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def cpu_baseline(w, max_seconds=20.0):
    """The CPU oracle on a bounded sample of the same workload: whole-grid
    steps of the 4096^2 disc until ~max_seconds of work (at least one)."""
    import oracle
    og = oracle.Grid(w.nx, w.ny, w.dx, w.dy, w.bcx, w.bcy, w.x0, w.y0, w.vc, w.rc)
    U = oracle.cons_field(w.W)
    t0 = time.perf_counter()
    steps = 0
    while True:
        dt = 0.8 / oracle.max_signal_speed(og, U)
        U = oracle.step(og, dt, U)
        steps += 1
        el = time.perf_counter() - t0
        if el > max_seconds or el / steps * (steps + 1) > max_seconds * 1.5:
            break
    threads = oracle.num_threads()
    return {"value": steps * w.nx * w.ny / el, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} whole-grid step(s) of the {w.nx}x{w.ny} disc (same input), "
                      f"{el:.1f} s, FP64 C oracle with {threads} OpenMP threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the sweep would shard by row slabs with a 2-row halo exchange; not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as wl
    import paper_1210_5246_amd as csh

    n, K, Wm = args.n, args.steps, args.warmup
    log(f"generating disc {n}^2")
    w = wl.disc(n, 3, K)
    cells = w.nx * w.ny

    def make(dtype):
        W = torch.from_numpy(w.W).to("cuda", dtype)
        g = csh.Grid(W, w.dx, w.dy, (w.bcx, w.bcy))
        g.set_potential(w.vc, w.rc, w.x0, w.y0)
        return g

    res = {}
    for name, dtype, bpc in (("f64", torch.float64, BYTES_PER_CELL_F64), ("f32", torch.float32, BYTES_PER_CELL_F32)):
        if name == "f32" and args.no_fp32:
            continue
        log(f"{name}: init + warmup")
        g = make(dtype)
        U0 = g.U.clone()
        if Wm > 0:
            g.run_cfl(Wm, 0.8)
        g.U.copy_(U0)
        g.run_cfl(K, 0.8)          # records the graph of K steps
        torch.cuda.synchronize()
        secs, dts = time_graph(g, U0, K)
        dt_first = float(dts[0].item())
        log(f"{name}: {K} steps in {secs * 1e3:.2f} ms")
        kern = time_kernel(g, U0, max(K, 10), dt_first)
        res[name] = {"secs": secs, "kernel_s": kern, "bpc": bpc}
        del g
        torch.cuda.empty_cache()

    f64 = res["f64"]
    value = K * cells / f64["secs"]
    achieved = f64["bpc"] * cells / f64["kernel_s"] / 1e9
    out = {
        "metric": "cell-updates/s (FP64 sweep, 4096^2 disc)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": f64["secs"] / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded disc-shaped input: exponential surface density, flat rotation curve, "
                "Toomre Q=1.5, anisotropic stress, m=2 perturbation)",
        "config": {"workload": f"disc {n}x{n}, FP64, {K} CFL steps at C=0.8, outflow, fixed potential",
                   "cells": cells, "rows_per_wave": None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sweep_kernel<double, 2-D>", "kernel_ms": f64["kernel_s"] * 1e3,
                     "algorithmic_bytes_per_launch": f64["bpc"] * cells},
    }
    if "f32" in res:
        f32 = res["f32"]
        out["fp32"] = {"value": K * cells / f32["secs"], "ms_per_step": f32["secs"] / K * 1e3,
                       "kernel_ms": f32["kernel_s"] * 1e3,
                       "achieved_GBs": f32["bpc"] * cells / f32["kernel_s"] / 1e9}
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

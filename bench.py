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
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_CELL_F64 = 96     # 6 conserved planes read + 6 written, 8 B each
BYTES_PER_CELL_F32 = 48
# Kurganov-Tadmor step, both stages in one launch (U* stays in registers):
# U read once, U^{n+1} written once
BYTES_PER_CELL_KT_F64 = 96
KT_CFL = 0.8
# 3-D: 10 planes read + 10 written = 160 B per cell-update for a single pass;
# the z-march also writes the two y-face states (160 B) and the partial update
# (80 B), which the second kernel reads back: 640 B
BYTES_PER_CELL_3D_MIN = 160
BYTES_PER_CELL_3D_DESIGN = 640
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector, published
VALU_ISSUE_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12  # lane-instructions per second, 1e12


PROFILES = os.path.join(ROOT, "profiles")
# the sweep kernel's sources and the file that sets its launch shape (rows per segment)
SWEEP_SOURCES = [os.path.join(ROOT, "paper_1210_5246_amd", "csrc", f)
                 for f in ("csh_fwd.hip", "csh_device.h", "csh_internal.h", "csh_api.hip")]


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_counters(n):
    """The committed rocprofv3 counter summary of the FP64 sweep (HBM bytes per
    launch, VALU counters), if it was taken on the current kernel sources."""
    path = os.path.join(PROFILES, f"sweep_disc{n}_f64_traffic.json")
    if not os.path.exists(path):
        return {}
    t = json.load(open(path))
    if t.get("kernel_source_hash") != sweep_source_hash():
        return {}
    return t


def valu_summary(t, kernel_s, cells):
    """FP64 VALU figures of the sweep beside its HBM roofline: the kernel sits
    near the FP64 VALU issue limit, which is what caps its bandwidth."""
    v = t.get("valu")
    if not v:
        return None
    tflops = v["fp64_flops_per_launch"] / kernel_s / 1e12
    # the ALU view: VALU lane-instructions issued per second against the issue
    # peak of 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64 instruction
    # per 4 cycles per SIMD)
    issue = v["valu_lane_instructions_per_cell"] * cells / kernel_s / 1e12
    return {"valu_busy": v["valu_busy"], "lane_instructions_per_cell": v["valu_lane_instructions_per_cell"],
            "fp64_flops_per_cell": v["fp64_flops_per_cell"], "fp64_tflops": tflops,
            "fp64_peak_tflops": FP64_PEAK_TFLOPS, "fp64_frac": tflops / FP64_PEAK_TFLOPS,
            "issue_tlane_instr_per_s": issue, "issue_peak_tlane_instr_per_s": VALU_ISSUE_PEAK_T,
            "issue_frac": issue / VALU_ISSUE_PEAK_T}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def time_graph(g, U0, steps, cfl=0.8):
    import torch
    g.U.copy_(U0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    dts = g.run_cfl(steps, cfl)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, dts


def time_kernel(g, U0, steps, dt):
    """Average duration of one csh_step (the sweep kernel alone; both stage
    kernels under the KT scheme): back-to-back launches on the handle's
    stream, bracketed by HIP events."""
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


def cpu_model() -> str:
    """The host CPU's model name (first entry of /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{steps} whole-grid step(s) of the {w.nx}x{w.ny} disc (same input), "
                      f"{el:.1f} s, FP64 C oracle with {threads} OpenMP threads"}


def bench_batched(steps=200):
    """512 uneven tubes x 200 steps: one persistent graph launch vs the plain
    path (per tube its own grid; per step a host round trip for the timestep
    and one launch)."""
    import numpy as np
    import torch
    import workloads as wl
    import paper_1210_5246_amd as csh
    t = wl.tubes(nsteps=steps)
    W = torch.from_numpy(t.W).to("cuda")
    b = csh.Batch(W, t.offsets)
    U0 = b.U.clone()
    best = b.autotune(probe_steps=8)
    b.run(steps, 0.8)                       # records the graph
    b.U.copy_(U0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.run(steps, 0.8)
    e1.record()
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) / 1e3
    Ub = b.U.cpu().numpy()
    log(f"batched: {t_batch * 1e3:.2f} ms (workgroup {best})")
    # plain path
    worst = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for k in range(t.lengths.size):
        n = int(t.lengths[k])
        g = csh.Grid(W[:, int(t.offsets[k]):int(t.offsets[k + 1])].contiguous(), 1.0 / n, 1.0,
                     (csh.BC_OUTFLOW, csh.BC_OUTFLOW))
        Ug = g.U
        for _ in range(steps):
            Ug = g.step(0.8 / g.max_signal_speed(Ug), Ug)
        outs.append(Ug)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for k, Ug in enumerate(outs):
        ref = Ug.cpu().numpy()
        got = Ub[:, int(t.offsets[k]):int(t.offsets[k + 1])]
        worst = max(worst, float(np.abs(got - ref).max() / np.abs(ref).max()))
    cells = int(t.offsets[-1]) * steps
    log(f"plain: {t_plain:.2f} s; max scaled difference {worst:.1e}")
    return {"workload": f"{t.lengths.size} tubes, lengths U{{128..4096}} (total {int(t.offsets[-1])} cells), "
                        f"{steps} steps, own CFL dt per tube, FP64",
            "batched_value": cells / t_batch, "plain_value": cells / t_plain, "unit": "cell-updates/s",
            "speedup": t_plain / t_batch, "batched_ms": t_batch * 1e3, "plain_s": t_plain,
            "workgroup": best, "max_scaled_difference": worst}


def bench_adjoint(n=512, steps=200, K=20, ndirs=64):
    """Gradient of 1/2 sum(rho_200 - rho*)^2 w.r.t. the initial fields: one
    checkpointed adjoint pass vs central differences on ndirs directions
    (2 ndirs forward runs at frozen timesteps)."""
    import torch
    import workloads as wl
    import paper_1210_5246_amd as csh
    from paper_1210_5246_amd import autograd as cag
    w0, wt = wl.adjoint(n, 5, 6, steps, K)
    Gt = csh.Grid(torch.from_numpy(wt.W).to("cuda"), wt.dx, wt.dy)
    Gt.run_cfl(steps, 0.8)
    rho_t = Gt.U[0].clone()
    Wd = torch.from_numpy(w0.W).to("cuda")

    def grad_once(k=K):
        W0 = Wd.clone().requires_grad_(True)
        U, dts = cag.sweep(W0, w0.dx, w0.dy, nsteps=steps, checkpoint_every=k)
        L = 0.5 * ((U[0] - rho_t) ** 2).sum()
        (gr,) = torch.autograd.grad(L, W0)
        return gr, dts

    grad_once()  # warm (graph capture, workspace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gr, dts = grad_once()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    # the same gradient with every state kept (checkpoint_every=1: one launch
    # sequence writes the trajectory, nothing is recomputed); bitwise equal
    grad_once(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gr1, _ = grad_once(1)
    torch.cuda.synchronize()
    t_grad_all = time.perf_counter() - t0
    same_all = bool(torch.equal(gr1, gr))
    del gr1
    g = csh.Grid(Wd, w0.dx, w0.dy)
    U0 = g.U.clone()
    g.run_cfl(steps, 0.8)
    g.U.copy_(U0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run_cfl(steps, 0.8)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    dirs = [torch.from_numpy(d).to("cuda") for d in wl.fd_directions(n, ndirs)]
    eps = 1e-6
    runner = cag.FrozenRunner(Wd, w0.dx, w0.dy, (0, 0), dts)
    runner.run(Wd)  # records the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fds = []
    for dd in dirs:
        rp = runner.run(Wd + eps * dd)[0].clone()
        rm = runner.run(Wd - eps * dd)[0]
        fds.append(float(((rp - rm) * (0.5 * (rp + rm) - rho_t)).sum()) / (2 * eps))
    torch.cuda.synchronize()
    t_fd = time.perf_counter() - t0
    worst = 0.0
    for dd, fd in zip(dirs, fds):
        gd = gr * dd
        worst = max(worst, abs(fd - float(gd.sum())) / float(gd.abs().sum()))
    log(f"adjoint: grad {t_grad:.3f} s, forward {t_fwd:.3f} s, FD({ndirs} dirs) {t_fd:.2f} s")
    return {"workload": f"periodic {n}x{n} FP64, {steps} steps, checkpoints every {K}, "
                        f"gradient vs central differences on {ndirs} directions (eps {eps})",
            "adjoint_gradient_s": t_grad, "forward_s": t_fwd, "fd_gradient_s": t_fd,
            "adjoint_gradient_s_all_states": t_grad_all, "all_states_gradient_bitwise_equal": same_all,
            "speedup": t_fd / t_grad, "adjoint_over_forward": t_grad / t_fwd,
            "max_fd_deviation_over_sum_abs_terms_eps1e-6": worst}


def bench_fourier(w, reps=20):
    """Global Fourier amplitudes A_1..A_6 of the 4096^2 disc's density: time
    per call (two kernels plus a 48-byte copy back), HBM bandwidth at 8 B/cell."""
    import torch
    import paper_1210_5246_amd as csh
    g = csh.Grid(torch.from_numpy(w.W).to("cuda"), w.dx, w.dy, (w.bcx, w.bcy))
    A = g.fourier_amplitudes(w.x0, w.y0, 6)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.fourier_amplitudes(w.x0, w.y0, 6)
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3 / reps
    cells = w.nx * w.ny
    return {"workload": f"A_1..A_6 of the {w.nx}x{w.ny} disc density (FP64)", "ms_per_call": secs * 1e3,
            "cells_per_s": cells / secs, "achieved_GBs": 8 * cells / secs / 1e9, "A": A}


def bench_3d(n=256, steps=10):
    """The 3-D ten-moment sweep on a periodic n^3 random state (FP64): graph-
    replayed device-timed steps; bandwidth at the design's bytes per cell."""
    import torch
    import workloads as wl
    import paper_1210_5246_amd as csh
    w = wl.periodic3(n, seed=7)
    G = csh.Grid3(torch.from_numpy(w.W).to("cuda"), w.h, w.bc)
    del w
    U0 = G.U.clone()
    G.run_cfl(steps, 0.8)                   # records the graph
    G.U.copy_(U0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    G.run_cfl(steps, 0.8)
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    cells = n ** 3
    return {"workload": f"periodic {n}^3 ten-moment state, FP64, {steps} CFL steps at C=0.8, HLL",
            "value": steps * cells / secs, "unit": "cell-updates/s", "ms_per_step": secs / steps * 1e3,
            "algorithmic_bytes_per_cell": BYTES_PER_CELL_3D_MIN,
            "design_bytes_per_cell": BYTES_PER_CELL_3D_DESIGN,
            "achieved_GBs_design": BYTES_PER_CELL_3D_DESIGN * cells * steps / secs / 1e9}


def copy_probe(nbytes=1 << 30):
    """A plain device copy of known size (for calibrating the HBM byte counters)."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy probe: {nbytes} bytes read + {nbytes} written per launch")


def device_copy_bandwidth(nbytes=1 << 30, reps=10):
    """Bytes moved per second (read + write) by a plain 1 GiB device-to-device
    copy, timed with HIP events: the practical HBM ceiling beside the
    8 TB/s published peak."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes * reps / secs / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-kt", action="store_true")
    ap.add_argument("--no-fourier", action="store_true")
    ap.add_argument("--no-hllc", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 1 GiB copy (counter calibration)")
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
    if args.copy_probe:
        copy_probe()
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
        res[name] = {"secs": secs, "kernel_s": kern, "bpc": bpc, "sim_t": float(dts.sum().item())}
        del g
        torch.cuda.empty_cache()

    copy_gbs = device_copy_bandwidth()
    log(f"device copy: {copy_gbs:.0f} GB/s")
    f64 = res["f64"]
    value = K * cells / f64["secs"]
    achieved = f64["bpc"] * cells / f64["kernel_s"] / 1e9
    counters = measured_counters(n)
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
                   "cells": cells},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counters.get("bytes_per_launch"),
                     "kernel": "sweep_kernel<double, 2-D>", "kernel_ms": f64["kernel_s"] * 1e3,
                     "kernel_source_hash": sweep_source_hash(),
                     "algorithmic_bytes_per_launch": f64["bpc"] * cells,
                     "valu": valu_summary(counters, f64["kernel_s"], cells),
                     "device_copy_GBs": copy_gbs, "frac_of_device_copy": achieved / copy_gbs,
                     # measured HBM bytes (the counters' traffic) per second of kernel time
                     "traffic_GBs": (counters["bytes_per_launch"] / f64["kernel_s"] / 1e9
                                     if counters.get("bytes_per_launch") else None)},
    }
    if "f32" in res:
        f32 = res["f32"]
        out["fp32"] = {"value": K * cells / f32["secs"], "ms_per_step": f32["secs"] / K * 1e3,
                       "kernel_ms": f32["kernel_s"] * 1e3,
                       "achieved_GBs": f32["bpc"] * cells / f32["kernel_s"] / 1e9}
    if not args.no_hllc:
        log("hllc: init + warmup")
        g = make(torch.float64)
        g.set_scheme("hllc")
        U0 = g.U.clone()
        if Wm > 0:
            g.run_cfl(Wm, 0.8)
        g.U.copy_(U0)
        g.run_cfl(K, 0.8)
        torch.cuda.synchronize()
        secs, dts = time_graph(g, U0, K)
        log(f"hllc: {K} steps in {secs * 1e3:.2f} ms")
        kern = time_kernel(g, U0, max(K, 10), float(dts[0].item()))
        out["hllc"] = {"value": K * cells / secs, "unit": "cell-updates/s", "ms_per_step": secs / K * 1e3,
                       "kernel_ms": kern * 1e3, "achieved_GBs": f64["bpc"] * cells / kern / 1e9,
                       "step_time_vs_hll": secs / f64["secs"]}
        del g
        torch.cuda.empty_cache()
    if not args.no_kt:
        log("kt: init + warmup")
        g = make(torch.float64)
        g.set_scheme("kt")
        U0 = g.U.clone()
        if Wm > 0:
            g.run_cfl(Wm, KT_CFL)
        g.U.copy_(U0)
        g.run_cfl(K, KT_CFL)
        torch.cuda.synchronize()
        secs, dts = time_graph(g, U0, K, KT_CFL)
        log(f"kt: {K} steps in {secs * 1e3:.2f} ms")
        kern = time_kernel(g, U0, max(K, 10), float(dts[0].item()))
        sim_t = float(dts.sum().item())
        out["kt"] = {"value": K * cells / secs, "unit": "cell-updates/s", "ms_per_step": secs / K * 1e3,
                     "kernel_ms_per_step": kern * 1e3, "launches_per_step": 1, "cfl": KT_CFL,
                     "achieved_GBs": BYTES_PER_CELL_KT_F64 * cells / kern / 1e9,
                     "step_time_vs_characteristic": secs / f64["secs"],
                     "sim_time_per_s": sim_t / secs,
                     "characteristic_sim_time_per_s": f64["sim_t"] / f64["secs"]}
        del g
        torch.cuda.empty_cache()
    if not args.no_fourier:
        log("fourier amplitudes")
        out["fourier"] = bench_fourier(w)
    if not args.no_3d:
        log("3-D sweep")
        out["sweep3d"] = bench_3d()
        torch.cuda.empty_cache()
    if not args.no_batch:
        log("batched tubes")
        out["batched"] = bench_batched()
    if not args.no_adjoint:
        log("adjoint gradient")
        out["adjoint"] = bench_adjoint()
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

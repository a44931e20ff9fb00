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
# a workgroup reads ten rows of 32 columns for six output rows of 28 columns,
# 80 x (10/6) x (32/28) = 152 B, unless the cache serves the overlap: 232 B
BYTES_PER_CELL_3D_MIN = 160
BYTES_PER_CELL_3D_DESIGN = 232
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


def _oracle_grid(w):
    import oracle
    return oracle.Grid(w.nx, w.ny, w.dx, w.dy, w.bcx, w.bcy, w.x0, w.y0, w.vc, w.rc)


def _oracle_steps(w, max_seconds, min_steps=1):
    """Whole-grid oracle CFL steps of workload w until ~max_seconds of work
    (at least min_steps): (steps, seconds)."""
    import oracle
    og = _oracle_grid(w)
    U = oracle.cons_field(w.W)
    t0 = time.perf_counter()
    steps = 0
    while True:
        dt = 0.8 / oracle.max_signal_speed(og, U)
        U = oracle.step(og, dt, U)
        steps += 1
        el = time.perf_counter() - t0
        if steps >= min_steps and (el > max_seconds or el / steps * (steps + 1) > max_seconds * 1.5):
            return steps, el


def cpu_baseline(w, seconds=(8.0, 4.0, 4.0)):
    """The CPU oracle (FP64 C, OpenMP over rows, never tuned) timed on bounded
    samples, in cell-updates/s.  The headline leg is the benchmark's own
    workload on all host threads; beside it the same workload on one thread
    (one step), the 1024^2 periodic workload (100 steps, extrapolated from a
    few) on all threads and on one, and the 512 uneven tubes (200 steps each,
    extrapolated from the first tubes)."""
    import oracle
    import workloads as wl
    threads = oracle.num_threads()
    legs = []
    steps, el = _oracle_steps(w, seconds[0])
    head = steps * w.nx * w.ny / el
    legs.append({"workload": f"disc {w.nx}x{w.ny}", "threads": threads, "value": head,
                 "sample": f"{steps} whole-grid step(s), {el:.1f} s"})
    oracle.set_num_threads(1)
    try:
        steps1, el1 = _oracle_steps(w, seconds[1])
    finally:
        oracle.set_num_threads(threads)
    legs.append({"workload": f"disc {w.nx}x{w.ny}", "threads": 1, "value": steps1 * w.nx * w.ny / el1,
                 "sample": f"{steps1} whole-grid step(s), {el1:.1f} s"})
    wp = wl.periodic(1024, 2, 100)
    for nth in (threads, 1):
        oracle.set_num_threads(nth)
        try:
            steps2, el2 = _oracle_steps(wp, seconds[2], min_steps=2)
        finally:
            oracle.set_num_threads(threads)
        legs.append({"workload": "periodic 1024x1024, 100 steps", "threads": nth,
                     "value": steps2 * wp.nx * wp.ny / el2,
                     "sample": f"{steps2} of the 100 steps, {el2:.1f} s; the 100-step run extrapolated to "
                               f"{100 * el2 / steps2:.1f} s at the same per-step cost"})
    t = wl.tubes(nsteps=200)
    t0 = time.perf_counter()
    done = cells = 0
    while done < t.lengths.size:
        wk = wl.tube_workload(t, done)
        og = oracle.Grid(wk.nx, 1, wk.dx, 1.0, wk.bcx, wk.bcy)
        oracle.run_cfl(og, oracle.cons_field(wk.W), nsteps=200)
        cells += wk.nx * 200
        done += 1
        if time.perf_counter() - t0 > seconds[2]:
            break
    el4 = time.perf_counter() - t0
    legs.append({"workload": f"{t.lengths.size} tubes x 200 steps", "threads": threads, "value": cells / el4,
                 "sample": f"the first {done} tubes ({cells // 200} cells) x 200 steps, {el4:.1f} s; all "
                           f"{t.lengths.size} tubes extrapolated to {el4 * int(t.offsets[-1]) * 200 / cells:.0f} s "
                           "at the same rate per cell-update"})
    return {"value": head, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{steps} whole-grid step(s) of the {w.nx}x{w.ny} disc (same input), {el:.1f} s, "
                      f"FP64 C oracle with {threads} OpenMP threads",
            "legs": legs}


def bench_batched(steps=200):
    """512 uneven tubes x 200 steps: one persistent graph launch against the
    plain one-grid-per-launch path.  The plain reference is each tube's own
    handle running its device-timed 200 steps as a replayed graph (handles and
    graphs made before the timed region, all tubes back to back on one
    stream); a host-stepped variant (per step a host round trip for the
    timestep and one launch) is reported beside it."""
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
    ntubes = t.lengths.size
    grids, starts, logs = [], [], []
    for k in range(ntubes):
        n = int(t.lengths[k])
        g = csh.Grid(W[:, int(t.offsets[k]):int(t.offsets[k + 1])].contiguous(), 1.0 / n, 1.0,
                     (csh.BC_OUTFLOW, csh.BC_OUTFLOW))
        starts.append(g.U.clone())
        logs.append(torch.empty(steps, dtype=torch.float64, device="cuda"))
        g.run_cfl(steps, 0.8, dt_log=logs[-1])   # records this handle's graph
        grids.append(g)
    for g, u0 in zip(grids, starts):
        g.U.copy_(u0)
    torch.cuda.synchronize()
    e0.record()
    for g, lg in zip(grids, logs):
        g.run_cfl(steps, 0.8, dt_log=lg)
    e1.record()
    torch.cuda.synchronize()
    t_plain = e0.elapsed_time(e1) / 1e3
    worst = 0.0
    for k, g in enumerate(grids):
        ref = g.U.cpu().numpy()
        got = Ub[:, int(t.offsets[k]):int(t.offsets[k + 1])]
        worst = max(worst, float(np.abs(got - ref).max() / np.abs(ref).max()))
    log(f"plain (graph per tube): {t_plain * 1e3:.1f} ms; max scaled difference {worst:.1e}")
    # host-stepped: max_signal_speed (a sync) and one step per launch
    for g, u0 in zip(grids, starts):
        g.U.copy_(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in grids:
        Ug = g.U
        for _ in range(steps):
            Ug = g.step(0.8 / g.max_signal_speed(Ug), Ug)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t0
    del grids
    cells = int(t.offsets[-1]) * steps
    log(f"plain (host-stepped): {t_host:.2f} s")
    return {"workload": f"{ntubes} tubes, lengths U{{128..4096}} (total {int(t.offsets[-1])} cells), "
                        f"{steps} steps, own CFL dt per tube, FP64",
            "batched_value": cells / t_batch, "plain_value": cells / t_plain, "unit": "cell-updates/s",
            "speedup": t_plain / t_batch, "batched_ms": t_batch * 1e3, "plain_ms": t_plain * 1e3,
            "plain": "per tube its own handle and a replayed graph of its 200 device-timed steps, "
                     "tubes back to back on one stream",
            "host_stepped_value": cells / t_host, "host_stepped_s": t_host,
            "speedup_vs_host_stepped": t_host / t_batch,
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
    # the same check at a smaller fixed step, where the differences cross
    # fewer limiter and tracing kinks (not timed)
    fds_small = []
    for dd in dirs:
        rp = runner.run(Wd + 1e-9 * dd)[0].clone()
        rm = runner.run(Wd - 1e-9 * dd)[0]
        fds_small.append(float(((rp - rm) * (0.5 * (rp + rm) - rho_t)).sum()) / 2e-9)
    worst, within, plain = 0.0, 0, []
    for dd, fd in zip(dirs, fds):
        gd = gr * dd
        ad = float(gd.sum())
        worst = max(worst, abs(fd - ad) / float(gd.abs().sum()))
        # the check's own measure: |FD - <grad, d>| <= 1e-5 max(|FD|, |<grad, d>|)
        rel = abs(fd - ad) / max(abs(fd), abs(ad))
        plain.append(rel)
        within += rel <= 1e-5
    within_small = sum(abs(fd - float((gr * dd).sum())) <= 1e-5 * max(abs(fd), abs(float((gr * dd).sum())))
                       for dd, fd in zip(dirs, fds_small))
    log(f"adjoint: grad {t_grad:.3f} s, forward {t_fwd:.3f} s, FD({ndirs} dirs) {t_fd:.2f} s; "
        f"{within}/{ndirs} directions within 1e-5")
    return {"workload": f"periodic {n}x{n} FP64, {steps} steps, checkpoints every {K}, "
                        f"gradient vs central differences on {ndirs} directions (eps {eps})",
            "adjoint_gradient_s": t_grad, "forward_s": t_fwd, "fd_gradient_s": t_fd,
            "adjoint_gradient_s_all_states": t_grad_all, "all_states_gradient_bitwise_equal": same_all,
            "speedup": t_fd / t_grad, "adjoint_over_forward": t_grad / t_fwd,
            "max_fd_deviation_over_sum_abs_terms_eps1e-6": worst,
            "fd_directions_within_1e-5": f"{within}/{ndirs}",
            "fd_relative_errors_eps1e-6": sorted(plain, reverse=True)[:4],
            "fd_relative_error_median_eps1e-6": sorted(plain)[len(plain) // 2],
            "fd_directions_within_1e-5_eps1e-9": f"{within_small}/{ndirs}"}


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

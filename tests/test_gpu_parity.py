"""Parity of the HIP sweep with the CPU oracle on seeded inputs.

Tolerances (FP64): max relative error (per-field metric of tests/parity.py)
<= 1e-12 after one step and <= 1e-10 after 100 steps.  Grid sizes span several
60-column strips and row segments with ragged tails; the full-size disc is
checked on sampled cells the oracle computes one by one.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import exact_riemann as er
import workloads as wl
import paper_1210_5246_amd as csh
from parity import max_rel_error

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL1 = 1e-12
TOL100 = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ogrid(w):
    return oracle.Grid(w.nx, w.ny, w.dx, w.dy, w.bcx, w.bcy, w.x0, w.y0, w.vc, w.rc)


def gpu_grid(w, dtype=torch.float64):
    W = torch.from_numpy(np.ascontiguousarray(w.W)).to(DEV, dtype)
    g = csh.Grid(W, w.dx, w.dy, (w.bcx, w.bcy))
    if w.vc:
        g.set_potential(w.vc, w.rc, w.x0, w.y0)
    return g


def rect_periodic(nx, ny, seed, bc=(0, 0)):
    n = max(nx, ny, 64)   # the smooth generator needs a few widths of room
    w = wl.periodic(n, seed)
    w.W = np.ascontiguousarray(w.W[:, :ny, :nx])
    w.nx, w.ny = nx, ny
    w.dx, w.dy = 1.0 / nx, 1.3 / ny
    w.bcx, w.bcy = bc
    return w


def test_init_state_matches_oracle():
    w = rect_periodic(250, 77, 21)
    say("init_state 250x77")
    g = gpu_grid(w)
    U = oracle.cons_field(w.W)
    # fused multiply-add on the GPU vs unfused in the oracle: a few ulp,
    # measured per field (Exy = Pxy + rho u v cancels towards zero)
    assert max_rel_error(g.U.cpu().numpy(), U) <= 1e-15


def test_nonphysical_input_is_rejected():
    w = rect_periodic(70, 20, 22)
    w.W[3, 5, 7] = -1.0
    say("nonphysical init")
    with pytest.raises(csh.NonPhysicalState):
        gpu_grid(w)


@pytest.mark.parametrize("cell", [(0, 0), (7, 59), (33, 60), (69, 129)])
def test_step_flags_a_nonphysical_result(cell):
    """A negative density slipped into a step's input makes its output
    non-finite around that cell; the sweep's fused validity test sets the
    handle's flag, which the next synchronising call reports, and set_state
    clears it."""
    w = rect_periodic(130, 70, 23)
    say("nonphysical step at", cell)
    g = gpu_grid(w)
    U = g.U.clone()
    U[0, cell[0], cell[1]] = -U[0, cell[0], cell[1]]
    g.step(1e-4, U)                         # asynchronous: no error yet
    with pytest.raises(csh.NonPhysicalState):
        g.last_signal_speed()
    g.set_state(torch.from_numpy(np.ascontiguousarray(w.W)).to(DEV))
    out = g.step(1e-4)
    assert torch.isfinite(out).all()
    assert g.last_signal_speed() > 0


@pytest.mark.parametrize("shape", [(250, 77), (61, 5), (7, 130), (1, 3)])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_one_step_2d(shape, bc):
    nx, ny = shape
    w = rect_periodic(nx, ny, 23, bc)
    say("one step 2d", shape, bc)
    g = gpu_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    s_o = oracle.max_signal_speed(og, U0)
    s_g = g.max_signal_speed()
    assert s_g == pytest.approx(s_o, rel=1e-14)
    dt = 0.8 / s_o
    ref = oracle.step(og, dt, U0)
    out = g.step(dt).cpu().numpy()
    assert max_rel_error(out, ref) <= TOL1
    # fused CFL rate of the output
    assert g.last_signal_speed() == pytest.approx(oracle.max_signal_speed(og, ref), rel=1e-13)


@pytest.mark.parametrize("rows", [1, 2, 3, 5])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (1, 0)])
def test_one_step_2d_short_segments(rows, bc, monkeypatch):
    """Row segments shorter than the march's two halo rows (the CSH_ROWS
    override, read when a handle is created): every segment edge is a
    boundary of the row rings."""
    w = rect_periodic(127, 23, 25, bc)
    say("one step 2d, rows per segment", rows, bc)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(og, U0)
    default = gpu_grid(w).step(dt).cpu().numpy()  # the library's own segment length
    monkeypatch.setenv("CSH_ROWS", str(rows))
    g = gpu_grid(w)
    out = g.step(dt).cpu().numpy()
    ref = oracle.step(og, dt, U0)
    assert max_rel_error(out, ref) <= TOL1
    # the same arithmetic per cell; which unrolled copy of the march loop takes a
    # row depends on where its segment starts, and the compiler may fuse the
    # multiply-adds of the copies differently: equal to rounding
    dev = max_rel_error(out, default)
    say("difference from the default segment length:", dev)
    assert dev <= 1e-14
    assert g.last_signal_speed() == pytest.approx(oracle.max_signal_speed(og, ref), rel=1e-13)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 59, 60, 61, 256, 1000])
@pytest.mark.parametrize("bc", [0, 1])
def test_one_step_1d(n, bc):
    w = wl.sod(max(n, 2))
    w.W = np.ascontiguousarray(wl.periodic(64, 24).W[:, 3, :].repeat(16, axis=1)[:, :n])
    w.nx, w.dx, w.bcx, w.bcy = n, 1.0 / n, bc, bc
    say("one step 1d", n, bc)
    g = gpu_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(og, U0)
    assert max_rel_error(g.step(dt).cpu().numpy(), oracle.step(og, dt, U0)) <= TOL1


def test_fluxes_match_oracle():
    w = rect_periodic(130, 70, 25, (1, 0))
    say("fluxes 130x70")
    g = gpu_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(og, U0)
    Fx_o, Fy_o = oracle.fluxes(og, dt, U0)
    Fx, Fy = g.fluxes(dt)
    for got, ref in ((Fx, Fx_o), (Fy, Fy_o)):
        got = got.cpu().numpy()
        scale = np.abs(ref).reshape(6, -1).max(axis=1)[:, None, None]
        assert (np.abs(got - ref) / scale).max() <= 1e-13


def test_hundred_steps_periodic_1024():
    """The 1024^2 periodic workload, 100 steps at CFL 0.8 with the timestep
    chosen on the device, against the oracle's own CFL loop."""
    w = wl.periodic(1024, 2, 100)
    say("periodic 1024^2 x 100 (oracle on CPU first)")
    og = ogrid(w)
    ref, dts_o = oracle.run_cfl(og, oracle.cons_field(w.W), nsteps=100, cfl=0.8)
    g = gpu_grid(w)
    dts = g.run_cfl(100, 0.8).cpu().numpy()
    np.testing.assert_allclose(dts, dts_o, rtol=1e-12)
    assert max_rel_error(g.U.cpu().numpy(), ref) <= TOL100


@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
def test_near_degenerate_stress_twenty_steps(bc):
    """A dynamically cold direction and a nearly singular stress tensor
    (Pyy / Pxx down to 1e-4, Pxy^2 up to 0.98 Pxx Pyy, the principal axes
    turning across the grid): the shear and fast speeds of the two directions
    differ by two orders of magnitude and q = Pxy / Pxx is large.  20 device-
    timed steps against the oracle's CFL loop."""
    nx, ny = 150, 70
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    pxx = 1.0 + 0.2 * np.cos(2 * np.pi * (X + Y))
    pyy = pxx * (1e-4 + 0.02 * (1 + np.sin(2 * np.pi * X)) ** 2)
    pxy = 0.99 * np.sqrt(pxx * pyy) * np.sin(2 * np.pi * (2 * X - Y))
    u = 0.3 * np.sin(2 * np.pi * Y)
    v = 0.05 * np.cos(2 * np.pi * X)
    W = np.ascontiguousarray(np.stack([rho, u, v, pxx, pxy, pyy]))
    say("near-degenerate stress 150x70 x 20, bc", bc)
    og = oracle.Grid(nx, ny, 1.0 / nx, 1.0 / ny, bc[0], bc[1])
    ref, dts_o = oracle.run_cfl(og, oracle.cons_field(W), nsteps=20, cfl=0.8)
    g = csh.Grid(torch.from_numpy(W).to(DEV), 1.0 / nx, 1.0 / ny, bc)
    dts = g.run_cfl(20, 0.8).cpu().numpy()
    np.testing.assert_allclose(dts, dts_o, rtol=1e-12)
    assert max_rel_error(g.U.cpu().numpy(), ref) <= TOL100
    assert g.last_signal_speed() > 0


def test_uniform_state_is_a_fixed_point():
    """A uniform moving state: every face sees the same two states and the
    flux differences vanish, so the state is a fixed point.  The kernel adds a
    cell's low y-face flux when it starts the cell's update and subtracts the
    equal high one a row later, (U + a) - a, which rounds: the state stays
    within a few units in the last place over ten device-timed steps (no
    potential), the same in every cell."""
    W = np.zeros((6, 33, 130))
    W[:] = np.array([1.3, 0.4, -0.2, 0.9, 0.1, 0.5])[:, None, None]
    g = csh.Grid(torch.from_numpy(W).to(DEV), 1.0 / 130, 1.0 / 33, (0, 0))
    U0 = g.U.clone()
    g.run_cfl(10, 0.8)
    err = float(((g.U - U0).abs() / U0.abs().clamp_min(1e-300)).max())
    say("uniform state, 10 steps, max relative change", err)
    assert err <= 1e-14
    assert torch.equal(g.U, g.U[:, :1, :1].expand_as(g.U))   # still uniform, bitwise


@pytest.mark.parametrize("axis", ["x", "y"])
def test_one_direction_profile_reduces_to_the_1d_sweep(axis):
    """Rows (columns) that are all the same: the y (x) slopes and the
    transverse terms vanish and the y (x) fluxes cancel exactly, so every row
    of the 2-D step is the 1-D step of the profile (with the axes exchanged
    for a profile along y), up to the rounding of the two kernels' multiply-
    add contractions."""
    n, m = 187, 9
    x = (np.arange(n) + 0.5) / n
    prof = np.stack([1.0 + 0.5 * np.tanh(20 * (x - 0.4)), 0.3 * np.sin(2 * np.pi * x), 0.1 * np.cos(2 * np.pi * x),
                     1.0 + 0.3 * np.sin(4 * np.pi * x), 0.2 * np.sin(2 * np.pi * x + 1), 0.8 + 0.1 * np.cos(6 * np.pi * x)])
    g1 = csh.Grid(torch.from_numpy(np.ascontiguousarray(prof[:, None, :])).to(DEV), 1.0 / n, 1.0, (1, 1))
    dt = 0.8 / g1.max_signal_speed()
    ref = g1.step(dt)[:, 0, :]
    if axis == "x":
        W = np.ascontiguousarray(np.repeat(prof[:, None, :], m, axis=1))
        g2 = csh.Grid(torch.from_numpy(W).to(DEV), 1.0 / n, 0.37, (1, 0))
        out = g2.step(dt)
        got = out
    else:
        swapped = prof[[0, 2, 1, 5, 4, 3]]       # (rho, v, u, Pyy, Pxy, Pxx): the profile along y
        W = np.ascontiguousarray(np.repeat(swapped[:, :, None], m, axis=2))
        g2 = csh.Grid(torch.from_numpy(W).to(DEV), 0.37, 1.0 / n, (0, 1))
        out = g2.step(dt)
        got = out[[0, 2, 1, 5, 4, 3]].transpose(1, 2)
    scale = ref.abs().amax(dim=1, keepdim=True)
    for k in range(m):
        err = float(((got[:, k, :] - ref).abs() / scale).max())
        assert err <= 1e-14, (k, err)


def test_host_dt_steps_equal_device_cfl_run():
    w = wl.periodic(192, 26, 12)
    say("host-dt loop vs device run_cfl")
    g1 = gpu_grid(w)
    U = g1.U.clone()
    dts = []
    s = g1.max_signal_speed(U)           # the device run also starts from this kernel
    for _ in range(12):
        dt = 0.8 / s
        U = g1.step(dt, U)
        dts.append(dt)
        s = g1.last_signal_speed()       # the rate the step fused, as the device run uses
        # the standalone reduction may contract differently: an ulp apart at most
        assert g1.max_signal_speed(U) == pytest.approx(s, rel=1e-15)
    g2 = gpu_grid(w)
    dts2 = g2.run_cfl(12, 0.8).cpu().numpy()
    np.testing.assert_allclose(dts2, dts, rtol=1e-15)
    assert torch.equal(U, g2.U)
    # replaying the captured graph from the same start gives the same answer
    g3 = gpu_grid(w)
    start = g3.U.clone()
    g3.run_cfl(12, 0.8)
    first = g3.U.clone()
    g3.U.copy_(start)
    g3.run_cfl(12, 0.8)
    assert torch.equal(first, g3.U)


def test_sod_tube_to_t02():
    """Sec. 4.1 tube, 256 cells, outflow, CFL 0.8 to t = 0.2 with the last step
    clipped on the device; against the oracle and the exact gamma = 3 solution."""
    w = wl.sod(256)
    say("sod 256 -> t=0.2")
    og = ogrid(w)
    ref, dts_o = oracle.run_cfl(og, oracle.cons_field(w.W), cfl=0.8, t_end=0.2)
    g = gpu_grid(w)
    dts = g.run_cfl(len(dts_o) + 7, 0.8, t_end=0.2).cpu().numpy()
    assert np.all(dts[len(dts_o):] == 0.0)
    np.testing.assert_allclose(dts[:len(dts_o)], dts_o, rtol=1e-12)
    U = g.U.cpu().numpy()
    assert max_rel_error(U, ref) <= TOL100
    assert np.all(U[2] == 0.0) and np.all(U[4] == 0.0)
    Wg = oracle.prim_field(U)
    ex = er.sod_bme_solution(w.extra["x"], 0.2)
    assert np.abs(Wg[0] - ex[0]).mean() < 6e-3


def test_disc_with_potential_full_grid_256():
    w = wl.disc(256, 3, 10)
    say("disc 256^2 x 10 with potential")
    og = ogrid(w)
    ref, dts_o = oracle.run_cfl(og, oracle.cons_field(w.W), nsteps=10)
    g = gpu_grid(w)
    dts = g.run_cfl(10, 0.8).cpu().numpy()
    np.testing.assert_allclose(dts, dts_o, rtol=1e-12)
    assert max_rel_error(g.U.cpu().numpy(), ref) <= 1e-11


def sample_cells(nx, ny, k, seed):
    r = np.random.default_rng(seed)
    cells = set(r.integers(0, nx * ny, size=k).tolist())
    for j in (0, 1, ny // 2, ny - 2, ny - 1):           # boundaries, strip and segment seams
        for i in (0, 1, 59, 60, 61, nx // 2, nx - 2, nx - 1):
            cells.add(j * nx + i)
    return np.array(sorted(cells), dtype=np.int64)


def test_disc_4096_one_step_sampled():
    """Full-size disc (4096^2, FP64, outflow, fixed potential): one step in the
    launch configuration of the benchmark, checked on sampled cells."""
    w = wl.disc(4096, 3, 1)
    say("disc 4096^2 one step, sampled")
    g = gpu_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    s = g.max_signal_speed()
    assert s == pytest.approx(oracle.max_signal_speed(og, U0), rel=1e-14)
    dt = 0.8 / s
    out = g.step(dt).cpu().numpy().reshape(6, -1)
    cells = sample_cells(4096, 4096, 3000, 31)
    ref = oracle.step_cells(og, dt, U0, cells).T
    assert max_rel_error(out[:, cells], ref) <= TOL1


def test_largest_fp64_grid_one_step_sampled():
    """The largest square FP64 grid the library accepts: 23170^2 = 536.8 M
    cells, one plane just under 4 GiB (byte offsets up to 4 GiB - 64 KiB),
    periodic; the 1024^2 periodic state tiled and cut, so the periodic wrap
    is a discontinuity.  One step against the oracle on sampled cells, among
    them the last rows and columns and the wrap."""
    n = 23170
    assert n * n * 8 < 1 << 32 <= (n + 1) * (n + 1) * 8
    base = wl.periodic(1024, 2)
    say("largest FP64 grid: tiling the input on the host")
    W = np.ascontiguousarray(np.tile(base.W, (1, 23, 23))[:, :n, :n])
    og = oracle.Grid(n, n, 1.0 / n, 1.0 / n, 0, 0)
    say("largest FP64 grid: device state")
    g = csh.Grid(torch.from_numpy(W).to(DEV), 1.0 / n, 1.0 / n, (0, 0))
    say("largest FP64 grid: oracle state and CFL rate")
    U0 = oracle.cons_field(W)
    del W
    s = g.max_signal_speed()
    assert s == pytest.approx(oracle.max_signal_speed(og, U0), rel=1e-14)
    dt = 0.8 / s
    say("largest FP64 grid: one step")
    out = g.step(dt)
    cells = set(sample_cells(n, n, 2000, 32).tolist())
    for j in (n - 3, n - 2, n - 1):                      # the last rows, the wrap in y
        for i in (0, 1, 59, 60, 61, n // 2, n - 3, n - 2, n - 1):
            cells.add(j * n + i)
    for j in (2, 1023, 1024, n // 2):                    # the last columns, the wrap in x
        for i in (n - 3, n - 2, n - 1):
            cells.add(j * n + i)
    cells = np.array(sorted(cells), dtype=np.int64)
    got = out.reshape(6, -1)[:, torch.from_numpy(cells).to(DEV)].cpu().numpy()
    say("largest FP64 grid: oracle on", cells.size, "cells")
    ref = oracle.step_cells(og, dt, U0, cells).T
    assert max_rel_error(got, ref) <= TOL1


def test_largest_fp32_grid_translation_invariant():
    """The largest square FP32 grid the library accepts: 32767^2 = 1.07 G
    cells, one plane just under 4 GiB (byte offsets up to 4 GiB - 128 KiB):
    the 1024^2 periodic state tiled and cut.  A property that holds at any
    size: away from the cut, every cell's update with a given dt is that of
    the same cell of the 1024^2 periodic grid with the same spacing (the
    scheme is translation invariant); the two agree to FP32 rounding (the
    unrolled copies of the row loop may fuse multiply-adds differently)."""
    n, m = 32767, 1024
    assert n * n * 4 < 1 << 32 <= (n + 1) * (n + 1) * 4
    base = wl.periodic(m, 2)
    small = csh.Grid(torch.from_numpy(base.W).to(DEV, torch.float32), 1.0 / n, 1.0 / n, (0, 0))
    dt = 0.8 / small.max_signal_speed()
    ref = small.step(dt).double()
    say("largest FP32 grid: tiling the input on the host")
    W = np.ascontiguousarray(np.tile(base.W.astype(np.float32), (1, 32, 32))[:, :n, :n])
    big = csh.Grid(torch.from_numpy(W).to(DEV), 1.0 / n, 1.0 / n, (0, 0))
    del W
    say("largest FP32 grid: one step")
    out = big.step(dt)
    r = np.random.default_rng(33)
    js = np.concatenate([r.integers(2, n - 2, 1500), [2, 3, m - 1, m, m + 1, n - 4, n - 3]])
    iss = np.concatenate([r.integers(2, n - 2, 1500), [n - 3, n - 4, 2, 59, 60, 61, n - 3]])
    flat = torch.from_numpy(js.astype(np.int64) * n + iss).to(DEV)
    got = out.reshape(6, -1)[:, flat].double()
    exp = ref.reshape(6, -1)[:, torch.from_numpy((js % m) * m + iss % m).to(DEV)]
    scale = exp.abs().amax(dim=1, keepdim=True)
    err = float(((got - exp).abs() / scale).max())
    say("largest FP32 grid: max difference from the 1024^2 grid", err)
    assert err <= 1e-6


def test_disc_4096_one_step_full():
    """Full-size disc (4096^2, FP64, outflow, fixed potential): one HLL step in
    the launch configuration of the benchmark against the oracle on every cell."""
    w = wl.disc(4096, 3, 1)
    say("disc 4096^2 one step, every cell (oracle ~5 s)")
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    g = gpu_grid(w)
    s = g.max_signal_speed()
    assert s == pytest.approx(oracle.max_signal_speed(og, U0), rel=1e-14)
    dt = 0.8 / s
    out = g.step(dt).cpu().numpy()
    ref = oracle.step(og, dt, U0)
    assert max_rel_error(out, ref) <= TOL1
    assert g.last_signal_speed() == pytest.approx(oracle.max_signal_speed(og, ref), rel=1e-13)


def test_disc_1024_fifty_steps_full_grid():
    """The disc workload at 1024^2 (outflow, fixed potential, kick after every
    step), 50 device-timed CFL steps against the oracle's own CFL loop on the
    whole grid: the timestep list to 1e-12 and the state to the 100-step bar."""
    w = wl.disc(1024, 3, 50)
    say("disc 1024^2 x 50 (oracle on CPU first, ~5-15 s)")
    og = ogrid(w)
    ref, dts_o = oracle.run_cfl(og, oracle.cons_field(w.W), nsteps=50, cfl=0.8)
    g = gpu_grid(w)
    dts = g.run_cfl(50, 0.8).cpu().numpy()
    np.testing.assert_allclose(dts, dts_o, rtol=1e-12)
    err = max_rel_error(g.U.cpu().numpy(), ref)
    say("disc 1024^2 x 50 max rel error:", err)
    assert err <= TOL100


def test_fp32_twin_close_to_fp64():
    """The FP32 instantiation on the disc shape: reported accuracy, loose bound."""
    w = wl.disc(512, 3, 5)
    say("fp32 disc 512^2 x 5")
    og = ogrid(w)
    ref, _ = oracle.run_cfl(og, oracle.cons_field(w.W), nsteps=5)
    g = gpu_grid(w, torch.float32)
    g.run_cfl(5, 0.8)
    err = max_rel_error(g.U.double().cpu().numpy(), ref)
    say("fp32 max rel error after 5 steps:", err)
    assert err < 1e-3


@pytest.mark.parametrize("scheme,shape", [("muscl", (130, 70)), ("kt", (130, 70)), ("kt", (300, 1)), ("hllc", (61, 5))])
def test_run_cfl_states_keeps_the_states_of_run_cfl(scheme, shape):
    """csh_run_cfl_states: every kept state and timestep is bitwise the one
    csh_run_cfl reaches after that many steps (disc-like potential on)."""
    nx, ny = shape
    w = rect_periodic(nx, max(ny, 2), 29, (1, 1))
    if ny == 1:
        w.W = np.ascontiguousarray(w.W[:, 0, :])
        w.ny, w.dy = 1, 1.0
    w.vc, w.rc, w.x0, w.y0 = 0.7, 0.1, -0.45, -0.5
    say("run_cfl_states", scheme, shape)
    g = gpu_grid(w)
    g.set_scheme(scheme)
    U0 = g.U.clone()
    states, dts = g.run_cfl_states(7, 0.8)
    assert torch.equal(g.U, U0)  # the initial state is only read
    for k in (0, 3, 6):
        r = gpu_grid(w)
        r.set_scheme(scheme)
        d = r.run_cfl(k + 1, 0.8)
        assert torch.equal(states[k], r.U), k
        assert torch.equal(dts[:k + 1], d), k


def test_run_dts_replays_run_cfl_bitwise_and_set_state():
    w = wl.periodic(200, 27, 9)
    say("run_dts replay")
    g = gpu_grid(w)
    W = torch.from_numpy(w.W).to(DEV)
    dts = g.run_cfl(9, 0.8).clone()
    ref = g.U.clone()
    g.set_state(W)                      # back to the initial state on the same handle
    g.run_dts(dts)
    assert torch.equal(g.U, ref)
    W2 = W.clone()
    W2[3, 4, 5] = -1.0
    with pytest.raises(csh.NonPhysicalState):
        g.set_state(W2)

"""Parity of the HIP Kurganov-Tadmor scheme (Sec. 3.2) with the oracle's.

Same bars as the characteristic sweep: max relative error (per-field metric of
tests/parity.py) <= 1e-12 after one step and <= 1e-10 after 100 steps, on
ragged shapes spanning several column strips (56 columns per wavefront in
2-D, 60 in 1-D) and row segments, around the strip edges, both boundary
kinds in each direction, 1-D and 2-D, with and without the external
potential; the full-size disc (4096^2) is compared on every cell after one
step.
"""
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


def kt_grid(w, dtype=torch.float64):
    W = torch.from_numpy(np.ascontiguousarray(w.W)).to(DEV, dtype)
    g = csh.Grid(W, w.dx, w.dy, (w.bcx, w.bcy))
    if w.vc:
        g.set_potential(w.vc, w.rc, w.x0, w.y0)
    g.set_scheme("kt")
    return g


def rect_periodic(nx, ny, seed, bc=(0, 0)):
    n = max(nx, ny, 64)
    w = wl.periodic(n, seed)
    w.W = np.ascontiguousarray(w.W[:, :ny, :nx])
    w.nx, w.ny = nx, ny
    w.dx, w.dy = 1.0 / nx, 1.3 / ny
    w.bcx, w.bcy = bc
    return w


@pytest.mark.parametrize("shape", [(250, 77), (61, 5), (7, 130), (1, 3), (2, 2), (56, 4), (57, 9), (113, 33)])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_kt_one_step_2d(shape, bc):
    nx, ny = shape
    w = rect_periodic(nx, ny, 41, bc)
    say("kt one step 2d", shape, bc)
    g = kt_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(og, U0)
    ref = oracle.step_kt(og, dt, U0)
    assert max_rel_error(g.step(dt).cpu().numpy(), ref) <= TOL1
    assert g.last_signal_speed() == pytest.approx(oracle.max_signal_speed(og, ref), rel=1e-13)


@pytest.mark.parametrize("rows", [1, 2, 3, 5])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_kt_short_segments(rows, bc, monkeypatch):
    """Row segments shorter than the fused march's halo (stage 1 runs 4 rows
    ahead of stage 2's owned rows; the CSH_KT_ROWS override, read at each
    launch): the ghost-row copies and the ring slots at every segment edge."""
    w = rect_periodic(127, 23, 43, bc)
    say("kt one step, rows per segment", rows, bc)
    g = kt_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(og, U0)
    default = g.step(dt).cpu().numpy()  # the library's own segment length
    monkeypatch.setenv("CSH_KT_ROWS", str(rows))
    out = g.step(dt).cpu().numpy()
    ref = oracle.step_kt(og, dt, U0)
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
def test_kt_one_step_1d(n, bc):
    w = wl.sod(max(n, 2))
    base = wl.periodic(64, 42).W[:, 3, :].repeat(16, axis=1)[:, :n]
    base[1] += 0.05 * np.sin(np.arange(n) * 0.7)   # n = 1, 2: a state that is not at rest
    w.W = np.ascontiguousarray(base)
    w.nx, w.dx, w.bcx, w.bcy = n, 1.0 / n, bc, bc
    say("kt one step 1d", n, bc)
    g = kt_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(og, U0)
    assert max_rel_error(g.step(dt).cpu().numpy(), oracle.step_kt(og, dt, U0)) <= TOL1


def test_kt_hundred_steps_periodic_512():
    """512^2 periodic, 100 device-timed CFL steps against the oracle's KT loop."""
    w = wl.periodic(512, 43, 100)
    say("kt periodic 512^2 x 100 (oracle first)")
    ref, dts_o = oracle.run_cfl(ogrid(w), oracle.cons_field(w.W), nsteps=100, cfl=0.8, scheme="kt")
    g = kt_grid(w)
    dts = g.run_cfl(100, 0.8).cpu().numpy()
    np.testing.assert_allclose(dts, dts_o, rtol=1e-12)
    assert max_rel_error(g.U.cpu().numpy(), ref) <= TOL100


def test_kt_host_dt_steps_equal_device_cfl_run_and_replay():
    w = wl.periodic(192, 44, 12)
    say("kt host-dt loop vs device run_cfl vs run_dts")
    g1 = kt_grid(w)
    U = g1.U.clone()
    dts = []
    s = g1.max_signal_speed(U)
    for _ in range(12):
        dt = 0.8 / s
        U = g1.step(dt, U)
        dts.append(dt)
        s = g1.last_signal_speed()
    g2 = kt_grid(w)
    dts2 = g2.run_cfl(12, 0.8).clone()
    np.testing.assert_allclose(dts2.cpu().numpy(), dts, rtol=1e-15)
    assert torch.equal(U, g2.U)
    g2.set_state(torch.from_numpy(w.W).to(DEV))
    g2.run_dts(dts2)
    assert torch.equal(U, g2.U)


def test_kt_sod_tube_to_t02():
    """The Sec. 4.1 tube under KT: oracle parity, the device-clipped last step,
    and the exact gamma = 3 solution (the bound of the oracle's own KT pin)."""
    w = wl.sod(256)
    say("kt sod 256 -> t=0.2")
    ref, dts_o = oracle.run_cfl(ogrid(w), oracle.cons_field(w.W), cfl=0.8, t_end=0.2, scheme="kt")
    g = kt_grid(w)
    dts = g.run_cfl(len(dts_o) + 5, 0.8, t_end=0.2).cpu().numpy()
    assert np.all(dts[len(dts_o):] == 0.0)
    np.testing.assert_allclose(dts[:len(dts_o)], dts_o, rtol=1e-12)
    U = g.U.cpu().numpy()
    assert max_rel_error(U, ref) <= TOL100
    assert np.all(U[2] == 0.0) and np.all(U[4] == 0.0)
    ex = er.sod_bme_solution(w.extra["x"], 0.2)
    assert np.abs(oracle.prim_field(U)[0] - ex[0]).mean() < 6e-3


def test_kt_disc_with_potential_256():
    w = wl.disc(256, 3, 10)
    say("kt disc 256^2 x 10 with potential")
    ref, dts_o = oracle.run_cfl(ogrid(w), oracle.cons_field(w.W), nsteps=10, cfl=0.8, scheme="kt")
    g = kt_grid(w)
    dts = g.run_cfl(10, 0.8).cpu().numpy()
    np.testing.assert_allclose(dts, dts_o, rtol=1e-12)
    assert max_rel_error(g.U.cpu().numpy(), ref) <= 1e-11


def test_kt_disc_4096_one_step_full():
    """Full-size disc (4096^2, FP64, outflow, potential): one KT step in the
    launch configuration of the benchmark against the oracle on every cell."""
    w = wl.disc(4096, 3, 1)
    say("kt disc 4096^2 one step (oracle ~5 s)")
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    g = kt_grid(w)
    dt = 0.8 / g.max_signal_speed()
    out = g.step(dt).cpu().numpy()
    assert max_rel_error(out, oracle.step_kt(og, dt, U0)) <= TOL1


def test_kt_fp32_close_to_fp64():
    w = wl.disc(512, 3, 5)
    say("kt fp32 disc 512^2 x 5")
    ref, _ = oracle.run_cfl(ogrid(w), oracle.cons_field(w.W), nsteps=5, cfl=0.8, scheme="kt")
    g = kt_grid(w, torch.float32)
    g.run_cfl(5, 0.8)
    err = max_rel_error(g.U.double().cpu().numpy(), ref)
    say("kt fp32 max rel error after 5 steps:", err)
    assert err < 1e-3


@pytest.mark.parametrize("shape,cell", [((130, 70), (0, 0)), ((130, 70), (37, 55)), ((130, 70), (69, 112)),
                                        ((200, 1), (0, 57))])
def test_kt_step_flags_a_nonphysical_result(shape, cell):
    """A negative density slipped into a KT step's input (2-D: the fused two-
    stage launch, around strip and segment seams; 1-D: the two launches) sets
    the handle's flag; the next synchronising call reports it."""
    w = rect_periodic(*shape, 24)
    say("kt nonphysical step", shape, cell)
    g = kt_grid(w)
    U = g.U.clone()
    U[0, cell[0], cell[1]] = -U[0, cell[0], cell[1]]
    g.step(1e-4, U)
    with pytest.raises(csh.NonPhysicalState):
        g.last_signal_speed()


def test_kt_rejects_characteristic_only_calls_and_switches_back():
    w = rect_periodic(70, 20, 45)
    say("kt scheme switching")
    g = kt_grid(w)
    U0 = g.U.clone()
    dt = 0.8 / g.max_signal_speed()
    with pytest.raises(csh.CshError):
        g.fluxes(dt)
    with pytest.raises(csh.CshError):
        g.adjoint_step(dt, U0, torch.ones_like(U0))
    kt = g.step(dt)
    g.set_scheme("muscl")
    og = ogrid(w)
    assert max_rel_error(g.step(dt).cpu().numpy(), oracle.step(og, dt, oracle.cons_field(w.W))) <= TOL1
    g.set_scheme("kt")
    assert torch.equal(g.step(dt), kt)

"""Parity of the HIP characteristic sweep with the HLLC flux against the
oracle's (reading H1), to the bars of the HLL sweep: max relative error
(per-field metric of tests/parity.py) <= 1e-12 after one step and <= 1e-10
after 100 steps, faces to 1e-13 of each field's scale, the full-size disc on
sampled cells and on every cell.  HLLC picks a side of the contact by the sign of S*; the flux is
continuous there, so a different pick on a rounding-level S* costs rounding."""
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


def hllc_grid(w, dtype=torch.float64):
    g = csh.Grid(torch.from_numpy(np.ascontiguousarray(w.W)).to(DEV, dtype), w.dx, w.dy, (w.bcx, w.bcy))
    if w.vc:
        g.set_potential(w.vc, w.rc, w.x0, w.y0)
    g.set_scheme("hllc")
    return g


def rect_periodic(nx, ny, seed, bc=(0, 0)):
    n = max(nx, ny, 64)
    w = wl.periodic(n, seed)
    w.W = np.ascontiguousarray(w.W[:, :ny, :nx])
    w.nx, w.ny = nx, ny
    w.dx, w.dy = 1.0 / nx, 1.3 / ny
    w.bcx, w.bcy = bc
    return w


@pytest.mark.parametrize("shape", [(250, 77), (61, 5), (7, 130), (1, 3)])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (0, 1)])
def test_hllc_one_step_2d(shape, bc):
    nx, ny = shape
    w = rect_periodic(nx, ny, 61, bc)
    say("hllc one step 2d", shape, bc)
    g = hllc_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(og, U0)
    ref = oracle.step(og, dt, U0, "hllc")
    assert max_rel_error(g.step(dt).cpu().numpy(), ref) <= TOL1
    assert g.last_signal_speed() == pytest.approx(oracle.max_signal_speed(og, ref), rel=1e-13)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 59, 60, 61, 256, 1000])
@pytest.mark.parametrize("bc", [0, 1])
def test_hllc_one_step_1d(n, bc):
    w = wl.sod(max(n, 2))
    base = wl.periodic(64, 62).W[:, 3, :].repeat(16, axis=1)[:, :n]
    base[1] += 0.05 * np.sin(np.arange(n) * 0.7)
    w.W = np.ascontiguousarray(base)
    w.nx, w.dx, w.bcx, w.bcy = n, 1.0 / n, bc, bc
    say("hllc one step 1d", n, bc)
    g = hllc_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(og, U0)
    assert max_rel_error(g.step(dt).cpu().numpy(), oracle.step(og, dt, U0, "hllc")) <= TOL1


def test_hllc_fluxes_match_oracle():
    w = rect_periodic(130, 70, 63, (1, 0))
    say("hllc fluxes 130x70")
    g = hllc_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(og, U0)
    Fx_o, Fy_o = oracle.fluxes(og, dt, U0, "hllc")
    Fx, Fy = g.fluxes(dt)
    for got, ref in ((Fx, Fx_o), (Fy, Fy_o)):
        got = got.cpu().numpy()
        scale = np.abs(ref).reshape(6, -1).max(axis=1)[:, None, None]
        assert (np.abs(got - ref) / scale).max() <= 1e-13


def test_hllc_hundred_steps_periodic_512():
    w = wl.periodic(512, 64, 100)
    say("hllc periodic 512^2 x 100 (oracle first)")
    ref, dts_o = oracle.run_cfl(ogrid(w), oracle.cons_field(w.W), nsteps=100, cfl=0.8, scheme="hllc")
    g = hllc_grid(w)
    dts = g.run_cfl(100, 0.8).cpu().numpy()
    np.testing.assert_allclose(dts, dts_o, rtol=1e-12)
    assert max_rel_error(g.U.cpu().numpy(), ref) <= TOL100


def test_hllc_host_dt_loop_equals_device_run():
    w = wl.periodic(192, 65, 12)
    say("hllc host-dt loop vs device run_cfl")
    g1 = hllc_grid(w)
    U = g1.U.clone()
    dts = []
    s = g1.max_signal_speed(U)
    for _ in range(12):
        dt = 0.8 / s
        U = g1.step(dt, U)
        dts.append(dt)
        s = g1.last_signal_speed()
    g2 = hllc_grid(w)
    np.testing.assert_allclose(g2.run_cfl(12, 0.8).cpu().numpy(), dts, rtol=1e-15)
    assert torch.equal(U, g2.U)


def test_hllc_sod_sharper_contact_than_hll():
    """Sec. 4.1 tube: oracle parity, exact solution, and on the GPU itself a
    density L1 error below the HLL sweep's."""
    w = wl.sod(256)
    say("hllc sod 256 -> t=0.2")
    ref, dts_o = oracle.run_cfl(ogrid(w), oracle.cons_field(w.W), cfl=0.8, t_end=0.2, scheme="hllc")
    g = hllc_grid(w)
    dts = g.run_cfl(len(dts_o) + 5, 0.8, t_end=0.2).cpu().numpy()
    np.testing.assert_allclose(dts[:len(dts_o)], dts_o, rtol=1e-12)
    U = g.U.cpu().numpy()
    assert max_rel_error(U, ref) <= TOL100
    ex = er.sod_bme_solution(w.extra["x"], 0.2)
    e_hllc = np.abs(oracle.prim_field(U)[0] - ex[0]).mean()
    gh = csh.Grid(torch.from_numpy(w.W).to(DEV), w.dx, 1.0, (w.bcx, w.bcy))
    gh.run_cfl(len(dts_o) + 5, 0.8, t_end=0.2)
    e_hll = np.abs(oracle.prim_field(gh.U.cpu().numpy())[0] - ex[0]).mean()
    say("density L1: hllc", e_hllc, "hll", e_hll)
    assert e_hllc < e_hll


def test_hllc_disc_with_potential_256():
    w = wl.disc(256, 3, 10)
    say("hllc disc 256^2 x 10")
    ref, dts_o = oracle.run_cfl(ogrid(w), oracle.cons_field(w.W), nsteps=10, scheme="hllc")
    g = hllc_grid(w)
    np.testing.assert_allclose(g.run_cfl(10, 0.8).cpu().numpy(), dts_o, rtol=1e-12)
    assert max_rel_error(g.U.cpu().numpy(), ref) <= 1e-11


def test_hllc_disc_4096_one_step_sampled():
    w = wl.disc(4096, 3, 1)
    say("hllc disc 4096^2 one step, sampled")
    g = hllc_grid(w)
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    dt = 0.8 / g.max_signal_speed()
    out = g.step(dt).cpu().numpy().reshape(6, -1)
    r = np.random.default_rng(66)
    cells = set(r.integers(0, 4096 * 4096, size=3000).tolist())
    for j in (0, 1, 2048, 4094, 4095):
        for i in (0, 1, 59, 60, 61, 2048, 4094, 4095):
            cells.add(j * 4096 + i)
    cells = np.array(sorted(cells), dtype=np.int64)
    ref = oracle.step_cells(og, dt, U0, cells, "hllc").T
    assert max_rel_error(out[:, cells], ref) <= TOL1


def test_hllc_disc_4096_one_step_full():
    """Full-size disc (4096^2, FP64, outflow, potential): one HLLC step in the
    launch configuration of the benchmark against the oracle on every cell."""
    w = wl.disc(4096, 3, 1)
    say("hllc disc 4096^2 one step, every cell (oracle ~5 s)")
    og = ogrid(w)
    U0 = oracle.cons_field(w.W)
    g = hllc_grid(w)
    dt = 0.8 / g.max_signal_speed()
    out = g.step(dt).cpu().numpy()
    assert max_rel_error(out, oracle.step(og, dt, U0, "hllc")) <= TOL1


def test_hllc_fp32_and_adjoint_refusal():
    w = wl.disc(512, 3, 5)
    say("hllc fp32 disc 512^2 x 5")
    ref, _ = oracle.run_cfl(ogrid(w), oracle.cons_field(w.W), nsteps=5, scheme="hllc")
    g = hllc_grid(w, torch.float32)
    g.run_cfl(5, 0.8)
    err = max_rel_error(g.U.double().cpu().numpy(), ref)
    say("hllc fp32 max rel error after 5 steps:", err)
    assert err < 1e-3
    g64 = hllc_grid(w)
    with pytest.raises(csh.CshError):
        g64.adjoint_step(1e-4, g64.U, torch.ones_like(g64.U))

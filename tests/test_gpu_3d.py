"""Parity of the HIP three-dimensional sweep (ten-moment system, HLL) with
the oracle's (cshoracle3.c), to the bars of the 2-D sweep: max relative error
per field (positive fields cell-wise, the others against the field's max
magnitude) <= 1e-12 after one step and <= 1e-10 after 30 steps; ragged
shapes, every boundary combination, degenerate extents (1 and 2 cells); the
128^3 workload on every cell after one step."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as wl
import paper_1210_5246_amd as csh

pytestmark = pytest.mark.gpu
DEV = "cuda"
POSITIVE = (0, 4, 7, 9)                  # rho, Exx, Eyy, Ezz


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(got, ref):
    worst = 0.0
    for m in range(10):
        g, r = got[m], ref[m]
        if m in POSITIVE:
            e = np.abs(g - r) / np.abs(r)
        else:
            e = np.abs(g - r) / max(np.abs(r).max(), np.abs(ref[1:4]).max(), 1e-300)
        worst = max(worst, float(e.max()))
    return worst


def workload(n, seed, bc=(0, 0, 0), h=None):
    nx, ny, nz = n
    w = wl.periodic3(nx, ny, nz, seed=seed, width=min(4.0, max(1.0, min(n) / 4)))
    h = h if h is not None else (1.0 / nx, 1.1 / ny, 0.9 / nz)
    return w.W, oracle.Grid3(nx, ny, nz, h[0], h[1], h[2], bc), h


def gpu(W, h, bc):
    return csh.Grid3(torch.from_numpy(np.ascontiguousarray(W)).to(DEV), h, bc)


@pytest.mark.parametrize("n", [(37, 29, 23), (61, 5, 7), (7, 64, 3), (1, 9, 11), (12, 1, 2), (2, 2, 2),
                               (9, 6, 1), (65, 3, 1), (28, 12, 5), (29, 13, 4)])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (0, 1, 0), (1, 0, 1)])
def test_3d_one_step(n, bc):
    W, g, h = workload(n, 71, bc)
    say("3d one step", n, bc)
    G = gpu(W, h, bc)
    U0 = oracle.cons3_field(W)
    s_o = oracle.max_signal_speed3(g, U0)
    assert G.max_signal_speed() == pytest.approx(s_o, rel=1e-13)
    dt = 0.8 / s_o
    ref = oracle.step3(g, dt, U0)
    assert rel_err(G.step(dt).cpu().numpy(), ref) <= 1e-12
    assert G.last_signal_speed() == pytest.approx(oracle.max_signal_speed3(g, ref), rel=1e-13)


@pytest.mark.parametrize("planes", [1, 2, 3])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1)])
def test_3d_short_segments(planes, bc, monkeypatch):
    """Runs of planes shorter than the sweep's halo planes (the CSH_PLANES
    override, read at each launch)."""
    W, g, h = workload((37, 11, 13), 73, bc)
    say("3d one step, planes per segment", planes, bc)
    G = gpu(W, h, bc)
    U0 = oracle.cons3_field(W)
    dt = 0.8 / oracle.max_signal_speed3(g, U0)
    default = G.step(dt).cpu().numpy()  # the library's own segment length
    monkeypatch.setenv("CSH_PLANES", str(planes))
    out = G.step(dt).cpu().numpy()
    ref = oracle.step3(g, dt, U0)
    assert rel_err(out, ref) <= 1e-12
    # the same arithmetic per cell; which unrolled copy of the plane loop takes a
    # row depends on where its segment starts, and the compiler may fuse the
    # multiply-adds of the copies differently: equal to rounding
    dev = rel_err(out, default)
    say("difference from the default segment length:", dev)
    assert dev <= 1e-14
    assert G.last_signal_speed() == pytest.approx(oracle.max_signal_speed3(g, ref), rel=1e-13)


@pytest.mark.parametrize("wg,planes", [(1, 0), (3, 0), (5, 0), (37, 0), (52, 0), (3, 2), (5, 3)])
def test_3d_workgroup_shares(wg, planes, monkeypatch):
    """The plane-columns dealt to other numbers of workgroups (the CSH_WG3
    override), alone and with runs capped at a few planes (CSH_PLANES). Here
    4 columns (2 strips x 2 row groups) of 13 planes: one or three
    workgroups take whole columns first and share the rest; five and more
    take only shares, which start and end inside a column and span columns;
    52 workgroups take one plane each."""
    bc = (0, 1, 0)
    W, g, h = workload((37, 11, 13), 78, bc)
    say("3d one step, workgroups", wg, "planes per run", planes or "all")
    G = gpu(W, h, bc)
    U0 = oracle.cons3_field(W)
    dt = 0.8 / oracle.max_signal_speed3(g, U0)
    default = G.step(dt).cpu().numpy()
    monkeypatch.setenv("CSH_WG3", str(wg))
    if planes:
        monkeypatch.setenv("CSH_PLANES", str(planes))
    out = G.step(dt).cpu().numpy()
    ref = oracle.step3(g, dt, U0)
    assert rel_err(out, ref) <= 1e-12
    dev = rel_err(out, default)
    say("difference from the default shares:", dev)
    assert dev <= 1e-14
    assert G.last_signal_speed() == pytest.approx(oracle.max_signal_speed3(g, ref), rel=1e-13)


def test_3d_thirty_steps_device_dt():
    W, g, h = workload((40, 36, 32), 72, (0, 1, 0))
    say("3d 40x36x32 x 30 (oracle first)")
    ref, dts_o = oracle.run_cfl3(g, oracle.cons3_field(W), 30)
    G = gpu(W, h, (0, 1, 0))
    dts = G.run_cfl(30, 0.8).cpu().numpy()
    np.testing.assert_allclose(dts, dts_o, rtol=1e-12)
    assert rel_err(G.U.cpu().numpy(), ref) <= 1e-10


def test_3d_host_loop_equals_device_run_and_replay():
    W, g, h = workload((24, 20, 16), 73)
    say("3d host loop vs device run vs replay")
    G1 = gpu(W, h, (0, 0, 0))
    U = G1.U.clone()
    s = G1.max_signal_speed(U)
    dts = []
    for _ in range(6):
        dt = 0.8 / s
        U = G1.step(dt, U)
        dts.append(dt)
        s = G1.last_signal_speed()
    G2 = gpu(W, h, (0, 0, 0))
    start = G2.U.clone()
    np.testing.assert_allclose(G2.run_cfl(6, 0.8).cpu().numpy(), dts, rtol=1e-15)
    assert torch.equal(U, G2.U)
    first = G2.U.clone()
    G2.U.copy_(start)
    G2.run_cfl(6, 0.8)                      # the recorded graph, replayed
    assert torch.equal(first, G2.U)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_3d_one_axis_profile_equals_the_thin_grid(axis):
    """A state that varies along one axis only: the slopes, transverse terms
    and flux differences of the two other axes vanish, so every line of a
    wide 3-D grid along that axis updates as the grid one cell thick in the
    other two (the same kernel: for y the workgroups' rows and their LDS
    exchange, for z the plane march, for x the lanes), up to the rounding of
    the order in which the update adds its flux differences."""
    n = 75
    t = (np.arange(n) + 0.5) / n
    prof = np.empty((10, n))
    prof[0] = 1.0 + 0.4 * np.tanh(15 * (t - 0.5))
    for k in range(1, 4):
        prof[k] = 0.2 * np.sin(2 * np.pi * t + k)
    # P = L L^T, L lower triangular with a positive diagonal: positive definite
    L = np.zeros((3, 3, n))
    L[0, 0], L[1, 1], L[2, 2] = 1.0 + 0.2 * np.sin(2 * np.pi * t), 0.8 + 0.1 * np.cos(4 * np.pi * t), 0.9 + 0.0 * t
    L[1, 0], L[2, 0], L[2, 1] = 0.3 * np.sin(2 * np.pi * t), 0.2 * np.cos(2 * np.pi * t), 0.1 * np.sin(6 * np.pi * t)
    P = np.einsum("ikn,jkn->ijn", L, L)
    for (i, j), m in zip(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)), range(4, 10)):
        prof[m] = P[i, j]
    h = (0.011, 0.013, 0.017)
    thin_shape = [1, 1, 1]
    thin_shape[axis] = n
    wide_shape = [6, 9, 5]
    wide_shape[axis] = n
    def field(shape):             # [10, nz, ny, nx] with the profile along the axis
        idx = [None, None, None]
        idx[2 - axis] = slice(None)
        return np.broadcast_to(prof[(slice(None),) + tuple(idx)], (10,) + tuple(shape[::-1])).copy()
    say("3d one-axis profile along", "xyz"[axis])
    bc_wide = [0, 0, 0]
    bc_wide[axis] = 1               # outflow along the profile, as on the thin grid
    bc_wide[(axis + 1) % 3] = 1     # and on one of the uniform axes
    Gt = gpu(field(thin_shape), h, (1, 1, 1))
    dt = 0.8 / Gt.max_signal_speed()
    ref = Gt.step(dt)
    Gw = gpu(field(wide_shape), h, tuple(bc_wide))
    out = Gw.step(dt)
    scale = ref.abs().reshape(10, -1).amax(dim=1).clamp_min(1e-300).view(10, 1, 1, 1)
    err = float(((out - ref.expand(out.shape)) / scale).abs().max())
    say("max difference from the thin grid", err)
    assert err <= 1e-14


def test_3d_128_full_grid():
    W, g, h = workload((128, 128, 128), 74, (1, 0, 0))
    say("3d 128^3 one step (oracle ~10 s)")
    G = gpu(W, h, (1, 0, 0))
    dt = 0.8 / G.max_signal_speed()
    out = G.step(dt).cpu().numpy()
    assert rel_err(out, oracle.step3(g, dt, oracle.cons3_field(W))) <= 1e-12


def test_3d_nonphysical_input_rejected():
    W, g, h = workload((8, 8, 8), 75)
    W[4, 3, 3, 3] = -1.0
    say("3d nonphysical init")
    with pytest.raises(csh.NonPhysicalState):
        gpu(W, h, (0, 0, 0))


@pytest.mark.parametrize("row", [0, 1, 2, 9, 10, 11, 13])
def test_3d_step_flags_a_nonphysical_result(row):
    """A negative density slipped into the input behind the handle's back
    makes the new state non-finite around it; the sweep's validity test (on
    whichever wavefront and half of its workgroup owns the row: the rows
    6k .. 6k + 5 of a group sit on the six output halves) raises the flag."""
    W, g, h = workload((20, 14, 10), 77)
    say("3d nonphysical step, row", row)
    G = gpu(W, h, (0, 1, 0))
    U = G.U.clone()
    U[0, 5, row, 9] = -U[0, 5, row, 9]
    with pytest.raises(csh.NonPhysicalState):
        G.step(1e-4, U)
    out = G.step(1e-4)                      # the handle still steps a valid state
    assert torch.isfinite(out).all()


def test_3d_256_benchmark_configuration():
    """The benchmark's state and launch configuration (periodic 256^3; 28-column
    strips, groups of six rows, the plane-columns dealt in equal shares to one
    workgroup per compute unit): one step compared cell by cell with the
    oracle on 3000 random cells plus cells on the strip and row-group seams,
    the periodic wrap and the planes where the shares of 256 workgroups (the
    MI355X's compute units: 256 whole columns, then shares of the other 174)
    start and end; then ten device-timed steps keep
    every conserved total to round-off (periodic boundaries: the face fluxes
    telescope)."""
    n = 256
    w = wl.periodic3(n, seed=7)
    say("3d 256^3 benchmark state: one step, sampled cells")
    G = gpu(w.W, w.h, w.bc)
    g = oracle.Grid3(n, n, n, w.h[0], w.h[1], w.h[2], w.bc)
    U0 = oracle.cons3_field(w.W)
    s_o = oracle.max_signal_speed3(g, U0)
    assert G.max_signal_speed() == pytest.approx(s_o, rel=1e-13)
    dt = 0.8 / s_o
    out = G.step(dt).cpu().numpy().reshape(10, -1)
    r = np.random.default_rng(76)
    cells = set(r.integers(0, n ** 3, size=3000).tolist())
    xs = (0, 1, 27, 28, 55, 56, 139, 140, 251, 252, 255)   # strips of 28 columns
    ys = (0, 5, 6, 11, 12, 127, 131, 132, 251, 252, 255)   # groups of 6 rows
    for x in xs:
        for y in ys:
            for z in (0, 1, 127, 128, 254, 255):
                cells.add((z * n + y) * n + x)
    strips, groups = (n + 27) // 28, (n + 5) // 6
    rest = (strips * groups - 256) * n                    # after 256 whole columns
    for k in range(0, 256, 9):                            # share boundaries
        col, z = divmod(256 * n + rest * k // 256, n)
        gy, sx = col % groups, col // groups
        for dz in (-1, 0):
            for x in (28 * sx, 28 * sx + 27):
                for y in (6 * gy, 6 * gy + 5):
                    if x < n and y < n:
                        cells.add((((z + dz) % n) * n + y) * n + x)
    cells = np.array(sorted(cells), dtype=np.int64)
    ref = oracle.step3_cells(g, dt, U0, cells).T          # [10, ncells]
    got = out[:, cells]
    scale = np.abs(U0.reshape(10, -1)).max(axis=1)
    for m in range(10):
        if m in POSITIVE:
            e = np.abs(got[m] - ref[m]) / np.abs(ref[m])
        else:
            e = np.abs(got[m] - ref[m]) / max(scale[m], scale[1:4].max())
        assert e.max() <= 1e-12, (m, float(e.max()))
    say("3d 256^3: ten device-timed steps, conservation")
    tot0 = U0.reshape(10, -1).sum(axis=1)
    mag = np.abs(U0.reshape(10, -1)).sum(axis=1)
    G.run_cfl(10, 0.8)
    tot1 = G.U.reshape(10, -1).sum(dim=1).cpu().numpy()
    assert np.all(np.abs(tot1 - tot0) <= 1e-12 * mag), (tot1 - tot0) / mag

"""The hand-written adjoint on the CPU (the kernels' per-cell bodies run in host
loops by tests/host/adjoint_host.hip): dot-product test against finite
differences of the same forward arithmetic, and the full transposed Jacobian
against the oracle's brute-force dense Jacobian on 8-cell grids."""
import ctypes
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "host"))
import build_host  # noqa: E402

_D = ctypes.POINTER(ctypes.c_double)
_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build_host.build())
        sig = [ctypes.c_int] * 4 + [ctypes.c_double] * 7 + [_D, _D, _D]
        L.host_adjoint_step.argtypes = sig
        L.host_adjoint_step_tiled.argtypes = sig
        L.host_step.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] * 7 + [_D, _D]
        L.host_init_adjoint.argtypes = [ctypes.c_int64, _D, _D, _D]
        L.host_xcd_block.argtypes = [ctypes.c_uint, ctypes.c_uint]
        L.host_xcd_block.restype = ctypes.c_uint
        _lib = L
    return _lib


def p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def geo(g):
    return (g.nx, g.ny, g.bcx, g.bcy, g.dx, g.dy)


def host_step(g, dt, U):
    out = np.empty_like(U)
    lib().host_step(*geo(g), dt, g.vc, g.rc, g.x0, g.y0, p(U), p(out))
    return out


def host_adjoint(g, dt, U, lam):
    out = np.empty_like(U)
    lib().host_adjoint_step(*geo(g), dt, g.vc, g.rc, g.x0, g.y0, p(U), p(np.ascontiguousarray(lam)), p(out))
    return out


def host_adjoint_tiled(g, dt, U, lam):
    """The tiled two-kernel reverse pass (2-D) run on the CPU."""
    out = np.empty_like(U)
    assert lib().host_adjoint_step_tiled(*geo(g), dt, g.vc, g.rc, g.x0, g.y0, p(U), p(np.ascontiguousarray(lam)),
                                         p(out)) == 0
    return out


def case(kind, bc):
    if kind == "2d":
        n = 10
        w = wl.periodic(64, 51)
        W = np.ascontiguousarray(w.W[:, 20:20 + n, 30:30 + n])
        W[1:3] *= 2.0
        g = oracle.Grid(n, n, 1.0 / n, 1.2 / n, bc, bc, -0.4, -0.55, 0.8 if bc else 0.0, 0.1)
    else:
        n = 12
        w = wl.periodic(64, 52)
        W = np.ascontiguousarray(w.W[:, 9, 10:10 + n])
        W[1] *= 2.0
        g = oracle.Grid(n, 1, 1.0 / n, 1.0, bc, bc, -0.3, 0.0, 0.6 if bc else 0.0, 0.2)
    U = oracle.cons_field(W)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    return g, U, dt


@pytest.mark.parametrize("kind", ["1d", "2d"])
@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_OUTFLOW])
def test_host_forward_matches_oracle(kind, bc):
    g, U, dt = case(kind, bc)
    ref = oracle.step(g, dt, U)
    got = host_step(g, dt, U)
    scale = np.abs(ref).reshape(6, -1).max(axis=1).reshape((6,) + (1,) * (U.ndim - 1))
    assert np.abs((got - ref) / scale).max() < 1e-13


@pytest.mark.parametrize("kind", ["1d", "2d"])
@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_OUTFLOW])
def test_dot_product_against_own_forward(kind, bc):
    """<lam, J d> by central differences of the same forward arithmetic equals
    <J^T lam, d> from the reverse pass."""
    g, U, dt = case(kind, bc)
    r = np.random.default_rng(7)
    for _ in range(4):
        lam = r.standard_normal(U.shape)
        d = r.standard_normal(U.shape) * np.abs(U).reshape(6, -1).max(axis=1).reshape((6,) + (1,) * (U.ndim - 1))
        eps = 1e-7
        Jd = (host_step(g, dt, U + eps * d) - host_step(g, dt, U - eps * d)) / (2 * eps)
        lhs = float((lam * Jd).sum())
        rhs = float((host_adjoint(g, dt, U, lam) * d).sum())
        assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), abs(rhs)), (lhs, rhs)


@pytest.mark.parametrize("kind", ["1d", "2d"])
@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_OUTFLOW])
def test_transposed_jacobian_matches_oracle_dense_jacobian(kind, bc):
    """Rows of J = d step / d U from the reverse pass (J^T e_k) against the
    oracle's central-difference dense Jacobian, 8 cells (1-D) / 8x8 (2-D)."""
    g, U, dt = case(kind, bc)
    if kind == "2d":
        g = oracle.Grid(8, 8, g.dx, g.dy, g.bcx, g.bcy, g.x0, g.y0, g.vc, g.rc)
        U = np.ascontiguousarray(U[:, :8, :8])
    else:
        g = oracle.Grid(8, 1, g.dx, 1.0, g.bcx, g.bcy, g.x0, 0.0, g.vc, g.rc)
        U = np.ascontiguousarray(U[:, :8])
    J = oracle.dense_jacobian(g, dt, U)
    n = U.size
    JT = np.empty((n, n))
    e = np.zeros(n)
    for k in range(n):
        e[:] = 0.0
        e[k] = 1.0
        JT[k, :] = host_adjoint(g, dt, U, e.reshape(U.shape)).ravel()   # J^T e_k = row k of J
    # per entry, the closer of two difference steps (a central difference that
    # straddles a limiter/HLL kink is not a derivative)
    J2 = oracle.dense_jacobian(g, dt, U, rel=1e-8)
    dev = np.minimum(np.abs(JT - J), np.abs(JT - J2)) / np.abs(J).max()
    assert dev.max() < 1e-6, dev.max()


def test_init_adjoint_is_transpose_of_cons():
    r = np.random.default_rng(3)
    W = wl.periodic(64, 53).W[:, :4, :5].copy()
    lamU = r.standard_normal(W.shape)
    d = r.standard_normal(W.shape)
    eps = 1e-7
    lhs = float((lamU * (oracle.cons_field(W + eps * d) - oracle.cons_field(W - eps * d)) / (2 * eps)).sum())
    out = np.empty_like(W)
    lib().host_init_adjoint(W[0].size, p(np.ascontiguousarray(W)), p(np.ascontiguousarray(lamU)), p(out))
    rhs = float((out * d).sum())
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs)


@pytest.mark.parametrize("nb", [1, 2, 7, 8, 9, 15, 16, 17, 1031, 1032, 1033])
def test_xcd_renumbering_is_a_bijection(nb):
    """The adjoint kernels' XCD-aware workgroup numbering covers every logical
    workgroup once, and hands each XCD (b % 8) one contiguous range."""
    f = lib().host_xcd_block
    logical = [f(b, nb) for b in range(nb)]
    assert sorted(logical) == list(range(nb))
    for x in range(8):
        mine = sorted(logical[b] for b in range(x, nb, 8))
        assert mine == list(range(mine[0], mine[0] + len(mine))) if mine else True


# grids around the tiles of the two-kernel reverse pass (A: 32 x 8 extended
# cells; B: 14 x 14 outputs) and tiny ones; every boundary combination
@pytest.mark.parametrize("shape", [(1, 4), (4, 2), (2, 2), (3, 5), (7, 3), (61, 6), (62, 7), (63, 13), (124, 12),
                                   (125, 31), (30, 9), (30, 14), (31, 15), (29, 13), (60, 28), (14, 14), (15, 15),
                                   (13, 29), (28, 43)])
@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_tiled_reverse_pass_equals_five_stage_pass(shape, bc):
    """The tiled reverse pass (wrap on periodic axes, folded ghost positions on
    outflow ones) against the five-stage pass on the extended grid: the same
    transpose, summed in another order."""
    nx, ny = shape
    w = wl.periodic(max(64, nx + 8, ny + 8), 53)
    W = np.ascontiguousarray(w.W[:, 3:3 + ny, 4:4 + nx])
    W[1:3] *= 2.0
    g = oracle.Grid(nx, ny, 1.0 / nx, 1.3 / ny, bc[0], bc[1], -0.45, -0.5, 0.7 if bc[0] else 0.0, 0.15)
    U = oracle.cons_field(W)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    lam = np.random.default_rng(nx * 100 + ny).standard_normal(U.shape)
    ref = host_adjoint(g, dt, U, lam)
    got = host_adjoint_tiled(g, dt, U, lam)
    assert np.all(np.isfinite(got))
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12

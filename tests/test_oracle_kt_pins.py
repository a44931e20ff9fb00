"""Pins of the oracle's Kurganov-Tadmor scheme (Sec. 3.2, eqs. (5)-(8)):
consistency and local speed of the numerical flux, the gamma = 3 Sod tube,
conservation, symmetry, and second-order convergence."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact_riemann as er
import workloads as wl
from test_oracle_pins import fd_jac, random_state, swap_xy


@pytest.mark.parametrize("direction", [0, 1])
def test_kt_flux_consistency_and_local_speed(direction):
    """H(w, w) = F(w); H(wl, wr) - (F(wl) + F(wr))/2 = -a/2 (U(wr) - U(wl)) with a
    the largest |eigenvalue| of dF/dU over the two states (eqs. (6)-(7))."""
    for _ in range(5):
        w = random_state()
        np.testing.assert_allclose(oracle.kt_flux(direction, w, w), oracle.flux(direction, oracle.cons(w)),
                                   rtol=1e-14, atol=1e-14)
        wl, wr = random_state(), random_state()
        H = oracle.kt_flux(direction, wl, wr)
        Ul, Ur = oracle.cons(wl), oracle.cons(wr)
        Fl, Fr = oracle.flux(direction, Ul), oracle.flux(direction, Ur)
        a = -2.0 * (H - 0.5 * (Fl + Fr)) / (Ur - Ul)
        rad = max(np.abs(np.linalg.eigvals(fd_jac(lambda x: oracle.flux(direction, x), U, 1e-3))).max()
                  for U in (Ul, Ur))
        np.testing.assert_allclose(a, rad, rtol=1e-7)


def run_sod(n, cfl=0.8):
    w = wl.sod(n)
    g = oracle.Grid(n, 1, 1.0 / n, 1.0, w.bcx, w.bcy)
    U, dts = oracle.run_cfl(g, oracle.cons_field(w.W), cfl=cfl, t_end=0.2, scheme="kt")
    return w, U, dts


def test_kt_sod_against_exact():
    w, U, dts = run_sod(256)
    dx = w.dx
    assert U[0].sum() * dx == pytest.approx(0.5625, abs=1e-14)
    assert U[3].sum() * dx == pytest.approx(0.55, abs=1e-14)
    assert U[5].sum() * dx == pytest.approx(0.55, abs=1e-14)
    assert U[1].sum() * dx == pytest.approx(0.9 * 0.2, abs=1e-14)
    assert np.all(U[2] == 0.0) and np.all(U[4] == 0.0)
    W = oracle.prim_field(U)
    ex = er.sod_bme_solution(w.extra["x"], 0.2)
    l1 = np.abs(W - ex).mean(axis=1)
    assert l1[0] < 6e-3 and l1[1] < 8e-3 and l1[3] < 5e-3


def test_kt_sod_converges():
    errs = []
    for n in (128, 256, 512):
        w, U, _ = run_sod(n)
        errs.append(np.abs(oracle.prim_field(U)[0] - er.sod_bme_solution(w.extra["x"], 0.2)[0]).mean())
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1]


@pytest.mark.parametrize("wave", [0, 2, 4])
def test_kt_linear_waves_second_order(wave):
    def err(n, eps=1e-6):
        w0 = np.array([1.0, 0.3, 0.1, 1.0, 0.2, 0.8])
        lam, R, _ = oracle.eigen(0, w0)
        x = (np.arange(n) + 0.5) / n
        W = w0[:, None] + eps * R[:, wave][:, None] * np.sin(2 * np.pi * x)[None, :]
        g = oracle.Grid(n, 1, 1.0 / n, 1.0)
        U, _ = oracle.run_cfl(g, oracle.cons_field(W), cfl=0.8, t_end=0.5, scheme="kt")
        Wex = w0[:, None] + eps * R[:, wave][:, None] * np.sin(2 * np.pi * (x - lam[wave] * 0.5))[None, :]
        return np.abs(oracle.prim_field(U) - Wex).mean() / eps
    e = [err(n) for n in (64, 128, 256)]
    assert math.log2(e[1] / e[2]) > 1.8, e


def test_kt_diagonal_wave_second_order():
    def err(n, eps=1e-6):
        c = (np.arange(n) + 0.5) / n
        X, Y = np.meshgrid(c, c)
        w0 = np.array([1.0, 0.6, 0.4, 1.0, 0.2, 0.7])
        W = np.broadcast_to(w0[:, None, None], (6, n, n)).copy()
        W[0] += eps * np.sin(2 * np.pi * (X + Y))
        g = oracle.Grid(n, n, 1.0 / n, 1.0 / n)
        U, _ = oracle.run_cfl(g, oracle.cons_field(W), cfl=0.8, t_end=0.25, scheme="kt")
        ex = w0[0] + eps * np.sin(2 * np.pi * (X - w0[1] * 0.25 + Y - w0[2] * 0.25))
        return np.abs(oracle.prim_field(U)[0] - ex).mean() / eps
    e = [err(n) for n in (32, 64, 128)]
    assert math.log2(e[1] / e[2]) > 1.8, e


def test_kt_conservation_free_stream_symmetry():
    w = wl.periodic(40, 71)
    U = oracle.cons_field(w.W)
    g = oracle.Grid(40, 40, w.dx, w.dy)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    U1 = oracle.step_kt(g, dt, U)
    scale = np.abs(U).reshape(6, -1).max(axis=1) * U[0].size
    assert np.all(np.abs(U1.reshape(6, -1).sum(axis=1) - U.reshape(6, -1).sum(axis=1)) <= 1e-13 * scale)
    np.testing.assert_allclose(oracle.step_kt(g, dt, swap_xy(U)), swap_xy(U1), rtol=1e-13, atol=1e-14)
    w0 = np.array([0.7, 0.3, -0.2, 0.5, 0.1, 0.9])
    Wc = np.broadcast_to(w0[:, None, None], (6, 16, 16)).copy()
    gc = oracle.Grid(16, 16, 1 / 16, 1 / 16, 1, 1)
    Uc = oracle.cons_field(Wc)
    np.testing.assert_allclose(oracle.step_kt(gc, 0.01, Uc), Uc, rtol=1e-14, atol=1e-15)

"""Pins of the oracle's HLLC flux for the BME (reading H1) and of the
characteristic scheme run with it (the solver of the paper's runs, Sec. 4.1).

What fixes the construction: consistency and upwinding; the three jump
conditions (across S_L, S* and S_R) and the fan average equal to the HLL
state; one velocity (S*, v*) in both star states; an isolated stationary or
moving contact (jumps in rho and the transverse stress only) kept exactly,
which HLL does not; the gamma = 3 Sod tube of Sec. 4.1 with a sharper contact
than HLL; conservation and second order on smooth waves.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact_riemann as er
import workloads as wl
from test_oracle_pins import random_state

rng = np.random.default_rng(11)


def swap(w):
    """Exchange the axes of a primitive or conserved 6-vector."""
    return np.array([w[0], w[2], w[1], w[5], w[4], w[3]])


@pytest.mark.parametrize("direction", [0, 1])
def test_consistency_and_upwinding(direction):
    n = 1 + direction
    for _ in range(10):
        w = random_state(rng)
        F = oracle.flux(direction, oracle.cons(w))
        np.testing.assert_allclose(oracle.hllc(direction, w, w), F, rtol=1e-13, atol=1e-13)
        fast = w.copy()
        fast[n] = 10.0                                   # supersonic to the right
        wr = random_state(rng)
        wr[n] = 10.0
        np.testing.assert_array_equal(oracle.hllc(direction, fast, wr), oracle.flux(direction, oracle.cons(fast)))
        fast[n] = wr[n] = -10.0
        np.testing.assert_array_equal(oracle.hllc(direction, fast, wr), oracle.flux(direction, oracle.cons(wr)))


@pytest.mark.parametrize("direction", [0, 1])
def test_jump_conditions_and_star_velocity(direction):
    n, t = (1, 2) if direction == 0 else (2, 1)
    for _ in range(20):
        wl_, wr_ = random_state(rng, 0.4), random_state(rng, 0.4)
        (sl, ss, sr), UsL, UsR = oracle.hllc_star(direction, wl_, wr_)
        assert sl < ss < sr
        Ul, Ur = oracle.cons(wl_), oracle.cons(wr_)
        Fl, Fr = oracle.flux(direction, Ul), oracle.flux(direction, Ur)
        FsL = Fl + sl * (UsL - Ul)                       # across S_L
        FsR = Fr + sr * (UsR - Ur)                       # across S_R
        scale = np.abs(np.concatenate([Fl, Fr, Ul, Ur])).max()
        np.testing.assert_allclose(FsR - FsL, ss * (UsR - UsL), atol=1e-13 * scale)   # across S*
        hll_state = (sr * Ur - sl * Ul - (Fr - Fl)) / (sr - sl)
        fan = ((ss - sl) * UsL + (sr - ss) * UsR) / (sr - sl)
        np.testing.assert_allclose(fan, hll_state, atol=1e-13 * scale)
        # one velocity in the star region
        for Us in (UsL, UsR):
            assert Us[n] / Us[0] == pytest.approx(ss, rel=1e-12, abs=1e-14)
        assert UsL[t] / UsL[0] == pytest.approx(UsR[t] / UsR[0], rel=1e-12, abs=1e-14)
        # the flux is the star flux on the side of the contact that holds x = 0
        F = oracle.hllc(direction, wl_, wr_)
        ref = Fl if sl >= 0 else FsL if ss >= 0 else FsR if sr > 0 else Fr
        np.testing.assert_allclose(F, ref, rtol=1e-13, atol=1e-13 * scale)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("u0", [0.0, 0.35, -0.35])
def test_isolated_contact_is_exact(direction, u0):
    """Jumps in rho and the transverse stress only (the two waves at speed u):
    HLLC returns the exact upwind flux, HLL diffuses the jump."""
    n = 1 + direction
    for _ in range(5):
        w0 = random_state(rng, 0.3)
        w0[n] = u0
        wl_, wr_ = w0.copy(), w0.copy()
        tt = 5 if direction == 0 else 3
        wl_[0], wr_[0] = 1.0, 0.3
        wl_[tt], wr_[tt] = 0.9 * w0[tt] + 0.05, 1.4 * w0[tt] + 0.05
        Fl = oracle.flux(direction, oracle.cons(wl_))
        Fr = oracle.flux(direction, oracle.cons(wr_))
        up = Fl if u0 >= 0 else Fr
        F = oracle.hllc(direction, wl_, wr_)
        np.testing.assert_allclose(F, up, rtol=1e-13, atol=1e-14)
        if u0 == 0.0:
            np.testing.assert_allclose(Fl, Fr, rtol=1e-14, atol=1e-14)
            assert abs(oracle.hll(direction, wl_, wr_)[0]) > 1e-3    # HLL moves mass across it


def test_axis_exchange():
    for _ in range(10):
        wl_, wr_ = random_state(rng), random_state(rng)
        np.testing.assert_allclose(oracle.hllc(1, swap(wl_), swap(wr_)), swap(oracle.hllc(0, wl_, wr_)),
                                   rtol=1e-14, atol=1e-14)


def run_sod(n, scheme):
    w = wl.sod(n)
    g = oracle.Grid(w.nx, 1, w.dx, 1.0, w.bcx, w.bcy)
    U, dts = oracle.run_cfl(g, oracle.cons_field(w.W), cfl=0.8, t_end=0.2, scheme=scheme)
    return w, U


def contact_width(W, ex):
    """Cells over which the density passes 5..95% of its jump at the contact."""
    jumps = np.where(np.abs(np.diff(ex[0])) > 0.02)[0]
    j = jumps[0]                                         # the contact (the shock is further right)
    lo, hi = ex[0][j], ex[0][j + 1]
    frac = (W[0][j - 20:j + 21] - lo) / (hi - lo)
    return int(((frac > 0.05) & (frac < 0.95)).sum())


def test_sod_tube_hllc():
    """The Sec. 4.1 tube (gamma = 3, 256 cells, t = 0.2): conservation, the
    exact solution, and a contact at least as sharp as HLL's."""
    w, U = run_sod(256, "hllc")
    dx = w.dx
    assert U[0].sum() * dx == pytest.approx(0.5625, abs=1e-14)
    assert U[3].sum() * dx == pytest.approx(0.55, abs=1e-14)
    assert U[5].sum() * dx == pytest.approx(0.55, abs=1e-14)
    assert U[1].sum() * dx == pytest.approx(0.9 * 0.2, abs=1e-14)
    assert np.all(U[2] == 0.0) and np.all(U[4] == 0.0)
    W = oracle.prim_field(U)
    ex = er.sod_bme_solution(w.extra["x"], 0.2)
    l1 = np.abs(W - ex).mean(axis=1)
    assert l1[0] < 5e-3 and l1[1] < 6e-3 and l1[3] < 4e-3
    _, Uh = run_sod(256, "muscl")
    Wh = oracle.prim_field(Uh)
    l1h = np.abs(Wh - ex).mean(axis=1)
    assert l1[0] < l1h[0] and l1[5] < l1h[5]
    assert contact_width(W, ex) <= contact_width(Wh, ex)


def test_sod_converges_hllc():
    errs = []
    for n in (128, 256, 512):
        w, U = run_sod(n, "hllc")
        errs.append(np.abs(oracle.prim_field(U)[0] - er.sod_bme_solution(w.extra["x"], 0.2)[0]).mean())
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1], errs


@pytest.mark.parametrize("wave", [0, 1, 2, 3, 4, 5])
def test_linear_waves_second_order_hllc(wave):
    def err(n, eps=1e-6):
        w0 = np.array([1.0, 0.3, 0.1, 1.0, 0.2, 0.8])
        lam, R, _ = oracle.eigen(0, w0)
        x = (np.arange(n) + 0.5) / n
        W = w0[:, None] + eps * R[:, wave][:, None] * np.sin(2 * np.pi * x)[None, :]
        g = oracle.Grid(n, 1, 1.0 / n, 1.0, oracle.BC_PERIODIC, oracle.BC_PERIODIC)
        U, _ = oracle.run_cfl(g, oracle.cons_field(W), cfl=0.8, t_end=0.5, scheme="hllc")
        Wex = w0[:, None] + eps * R[:, wave][:, None] * np.sin(2 * np.pi * (x - lam[wave] * 0.5))[None, :]
        return np.abs(oracle.prim_field(U) - Wex).mean() / eps
    e = [err(n) for n in (64, 128, 256)]
    assert math.log2(e[1] / e[2]) > 1.75, e


def test_periodic_conservation_and_transpose_2d():
    w = wl.periodic(48, 7)
    g = oracle.Grid(48, 40, 1.0 / 48, 1.1 / 40)
    W = np.ascontiguousarray(w.W[:, :40, :48])
    U = oracle.cons_field(W)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    U1 = oracle.step(g, dt, U, "hllc")
    np.testing.assert_allclose(U1.reshape(6, -1).sum(axis=1), U.reshape(6, -1).sum(axis=1), rtol=1e-13, atol=1e-12)
    gt = oracle.Grid(40, 48, 1.1 / 40, 1.0 / 48)
    Ut = np.ascontiguousarray(np.stack([U[0], U[2], U[1], U[5], U[4], U[3]]).transpose(0, 2, 1))
    U1t = oracle.step(gt, dt, Ut, "hllc")
    back = np.stack([U1t[0], U1t[2], U1t[1], U1t[5], U1t[4], U1t[3]]).transpose(0, 2, 1)
    np.testing.assert_allclose(back, U1, rtol=1e-12, atol=1e-13)

"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: velocity
moments of a distribution function (the definition of the moment equations,
Sec. 2), a finite-difference Jacobian of its own conservative flux, textbook
exact Riemann solutions, exact conservation integrals, closed forms of the
gamma = 3 rarefaction, symmetries and convergence orders.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import exact_riemann as er
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.default_rng(12345)


def random_state(g=rng, umax=1.0):
    rho = math.exp(0.5 * g.standard_normal())
    u, v = umax * g.standard_normal(2)
    L = np.array([[0.5 + g.random(), 0.0], [g.uniform(-0.5, 0.5), 0.5 + g.random()]])
    P = rho * L @ L.T
    return np.array([rho, u, v, P[0, 0], P[0, 1], P[1, 1]])


def sigma_points(w):
    """A symmetric discrete velocity distribution (zero third central moment)
    with density rho, mean (u, v) and dispersion P / rho."""
    rho, u, v = w[0], w[1], w[2]
    S = np.array([[w[3], w[4]], [w[4], w[5]]]) / rho
    C = np.linalg.cholesky(S)
    pts = []
    for k in range(2):
        for s in (1.0, -1.0):
            pts.append(np.array([u, v]) + s * math.sqrt(2.0) * C[:, k])
    return np.array(pts), np.full(4, rho / 4.0)


def moments(pts, wt, weight):
    vx, vy = pts[:, 0], pts[:, 1]
    return np.array([(wt * weight * q).sum() for q in (np.ones_like(vx), vx, vy, vx * vx, vx * vy, vy * vy)])


# ---- Sec. 2: variables and fluxes are velocity moments ---------------------------------

@pytest.mark.parametrize("trial", range(8))
def test_conserved_and_flux_are_velocity_moments(trial):
    """U = int m (1, v, v v) f dv and F_k = int m v_k (1, v, v v) f dv for any f with
    Q_ijk = 0 (Sec. 2, eqs. (2)-(4) and the moment definitions before them)."""
    w = random_state()
    pts, wt = sigma_points(w)
    U = oracle.cons(w)
    np.testing.assert_allclose(U, moments(pts, wt, 1.0), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle.flux(0, U), moments(pts, wt, pts[:, 0]), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(oracle.flux(1, U), moments(pts, wt, pts[:, 1]), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(oracle.prim(U), w, rtol=1e-13, atol=1e-14)


# ---- Sec. 3.3: eigen-system ---------------------------------------------------------------

def fd_jac(f, x, h):
    x = np.asarray(x, float)
    cols = []
    for k in range(x.size):
        e = np.zeros_like(x); e[k] = h * max(1.0, abs(x[k]))
        # 4th-order central difference
        d = (-f(x + 2 * e) + 8 * f(x + e) - 8 * f(x - e) + f(x - 2 * e)) / (12 * e[k])
        cols.append(d)
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("trial", range(6))
def test_primitive_jacobian_matches_conservative_flux(direction, trial):
    """A_W = M^-1 (dF/dU) M, M = dU/dW: the quasi-linear form used for tracing is
    the conservative flux of eqs. (2)-(4) (reading R2; the printed eq. (16)
    misses rho at (1,2) and the transverse compression terms)."""
    w = random_state()
    U = oracle.cons(w)
    dFdU = fd_jac(lambda x: oracle.flux(direction, x), U, 1e-3)
    M = fd_jac(oracle.cons, w, 1e-3)
    AW = np.linalg.solve(M, dFdU @ M)
    np.testing.assert_allclose(oracle.jacobian(direction, w), AW, rtol=1e-8, atol=1e-8)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("trial", range(6))
def test_eigensystem(direction, trial):
    """A R = R Lambda and L R = I (eqs. (14), (17), (18), extended to the full tensor)."""
    w = random_state()
    A = oracle.jacobian(direction, w)
    lam, R, L = oracle.eigen(direction, w)
    scale = np.abs(A).max() * np.abs(R).max()
    assert np.abs(A @ R - R @ np.diag(lam)).max() <= 1e-14 * scale * 8
    assert np.abs(L @ R - np.eye(6)).max() <= 1e-13
    # eigenvalues of the conservative Jacobian: u_n -+ a, u_n -+ c, u_n, u_n
    U = oracle.cons(w)
    ev = np.sort(np.linalg.eigvals(fd_jac(lambda x: oracle.flux(direction, x), U, 1e-3)).real)
    un, pnn = (w[1], w[3]) if direction == 0 else (w[2], w[5])
    a, c = math.sqrt(3 * pnn / w[0]), math.sqrt(pnn / w[0])
    np.testing.assert_allclose(ev, np.sort([un - a, un - c, un, un, un + c, un + a]), atol=1e-7)
    np.testing.assert_allclose(np.sort(lam), np.sort([un - a, un - c, un, un, un + c, un + a]), rtol=1e-14)


def test_eigensystem_reduces_to_paper_for_diagonal_stress():
    """For Pxy = 0 the fast waves (u -+ a) and the density wave are those of
    eqs. (17)-(18) restricted to 2-D: r = (rho, -+a, 0, rho a^2, 0, Pyy)... the
    paper's 7-variable columns have Pyy = 0 in the fast vectors because its
    eq. (16) drops the Pyy u_x term; the rho, u, Pxx entries must agree."""
    w = np.array([1.3, 0.2, -0.1, 0.9, 0.0, 0.5])
    lam, R, L = oracle.eigen(0, w)
    a = math.sqrt(3 * w[3] / w[0])
    np.testing.assert_allclose(lam[[0, 5]], [w[1] - a, w[1] + a], rtol=1e-15)
    np.testing.assert_allclose(R[[0, 1, 3], 0], [w[0], -a, w[0] * a * a], rtol=1e-14)
    np.testing.assert_allclose(R[[0, 1, 3], 5], [w[0], a, w[0] * a * a], rtol=1e-14)
    np.testing.assert_allclose(L[0, [1, 3]], [-1 / (2 * a), 1 / (2 * w[0] * a * a)], rtol=1e-14)
    np.testing.assert_allclose(L[5, [1, 3]], [1 / (2 * a), 1 / (2 * w[0] * a * a)], rtol=1e-14)
    np.testing.assert_allclose(L[2, [0, 3]], [1.0, -1 / (a * a)], rtol=1e-14)


# ---- eq. (25): MC limiter ------------------------------------------------------------------

@pytest.mark.parametrize("dl,dc,dr,expect", [
    (1.0, 1.0, 1.0, 1.0),          # smooth: centred difference
    (1.0, 2.0, 3.0, 2.0),          # centred is smallest
    (0.2, 1.1, 2.0, 0.4),          # 2|dl| binds
    (2.0, 1.1, 0.2, 0.4),          # 2|dr| binds
    (-1.0, -2.0, -3.0, -2.0),      # negative slopes keep their sign
    (-0.1, -1.0, -3.0, -0.2),
    (1.0, 0.0, -1.0, 0.0),         # extremum: zero (reading R3)
    (0.0, 0.5, 1.0, 0.0),          # flat on one side: zero
    (-2.0, 0.5, 3.0, 0.0),
])
def test_mc_truth_table(dl, dc, dr, expect):
    assert oracle.mc(dl, dc, dr) == pytest.approx(expect, abs=0, rel=1e-15)


# ---- HLL ----------------------------------------------------------------------------------

@pytest.mark.parametrize("direction", [0, 1])
def test_hll_consistency_and_upwinding(direction):
    for _ in range(5):
        w = random_state()
        U = oracle.cons(w)
        np.testing.assert_allclose(oracle.hll(direction, w, w), oracle.flux(direction, U),
                                   rtol=1e-13, atol=1e-14)
    # supersonic to the right: HLL is the left flux
    wl, wr = random_state(), random_state()
    iv, ip = (1, 3) if direction == 0 else (2, 5)
    wl[iv] = 5.0 + math.sqrt(3 * wl[ip] / wl[0])
    wr[iv] = 5.0 + math.sqrt(3 * wr[ip] / wr[0])
    np.testing.assert_array_equal(oracle.hll(direction, wl, wr), oracle.flux(direction, oracle.cons(wl)))
    wl[iv] = -wl[iv]; wr[iv] = -wr[iv]
    np.testing.assert_array_equal(oracle.hll(direction, wl, wr), oracle.flux(direction, oracle.cons(wr)))


# ---- eqs. (27)-(32): tracing ----------------------------------------------------------------

@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("umean", [0.0, 3.0, -3.0, 0.4])
def test_trace_sums_each_wave_once(direction, umean):
    """With the HLL terms added (reading R5) the per-wave sums collapse, since
    sum_a lam_a (l_a.dw) r_a = A dw and sum_a (l_a.dw) r_a = dw, to
      w_hi = w + dw/2 - k A dw + k min(lamM, 0) dw
      w_lo = w - dw/2 - k A dw + k max(lam0, 0) dw
    for every sign pattern of the eigenvalues (sub- and supersonic)."""
    for _ in range(5):
        w = random_state(umax=0.3)
        w[1 + direction] += umean
        dw = 0.1 * rng.standard_normal(6)
        k = 0.37
        lo, hi = oracle.trace(direction, w, dw, k)
        A = oracle.jacobian(direction, w)
        lam, _, _ = oracle.eigen(direction, w)
        hi_cf = w + 0.5 * dw - k * A @ dw + k * min(lam.max(), 0.0) * dw
        lo_cf = w - 0.5 * dw - k * A @ dw + k * max(lam.min(), 0.0) * dw
        np.testing.assert_allclose(hi, hi_cf, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(lo, lo_cf, rtol=1e-12, atol=1e-13)


def test_trace_continuous_at_zero_speed():
    """A contact wave with speed exactly 0 (the Sod initial state) is traced as
    its neighbours at speeds +-tiny are: the face states are continuous."""
    w = np.array([1.0, 0.0, 0.0, 1.0, 0.1, 0.8])
    dw = np.array([0.1, 0.05, -0.02, 0.3, 0.01, -0.2])
    lo0, hi0 = oracle.trace(0, w, dw, 0.4)
    for eps in (1e-300, -1e-300):
        w2 = w.copy(); w2[1] = eps
        lo, hi = oracle.trace(0, w2, dw, 0.4)
        np.testing.assert_allclose(lo, lo0, rtol=1e-15, atol=1e-16)
        np.testing.assert_allclose(hi, hi0, rtol=1e-15, atol=1e-16)


# ---- exact Riemann solver -----------------------------------------------------------------

def test_exact_solver_textbook_sod():
    gold = json.load(open(os.path.join(GOLDEN, "sod_gamma14_toro.json")))
    L = er.State(gold["left"]["rho"], gold["left"]["u"], gold["left"]["p"])
    R = er.State(gold["right"]["rho"], gold["right"]["u"], gold["right"]["p"])
    p, u = er.star_state(L, R, gold["gamma"])
    rl, rr = er.star_densities(L, R, gold["gamma"])
    tol = 0.5 * 10.0 ** (-gold["digits"])
    s = gold["star"]
    assert abs(p - s["p"]) <= tol and abs(u - s["u"]) <= tol
    assert abs(rl - s["rho_left"]) <= tol and abs(rr - s["rho_right"]) <= tol


def test_exact_solver_gamma3_closed_forms():
    """gamma = 3: Rankine-Hugoniot at the shock, isentropic star-left state and
    the linear rarefaction fan u = (a_L + xi)/2, a = (a_L - xi)/2, rho ~ a, p ~ rho^3."""
    gold = json.load(open(os.path.join(GOLDEN, "sod_bme_setup.json")))
    L = er.State(gold["left"]["rho"], gold["left"]["u"], gold["left"]["Pxx"])
    R = er.State(gold["right"]["rho"], gold["right"]["u"], gold["right"]["Pxx"])
    g = 3.0
    p, u = er.star_state(L, R, g)
    rl, rr = er.star_densities(L, R, g)
    S = er.wave_speeds(L, R, g)["right_shock"]
    # RH: mass, momentum, energy fluxes continuous in the shock frame
    def fluxes(rho, uu, pp):
        m = rho * (uu - S)
        e = pp / (g - 1) + 0.5 * rho * uu * uu
        return np.array([m, m * uu + pp, (e + pp) * uu - S * e])
    np.testing.assert_allclose(fluxes(rr, u, p), fluxes(R.rho, R.u, R.p), rtol=1e-12, atol=1e-12)
    assert rl == pytest.approx(L.rho * (p / L.p) ** (1 / g), rel=1e-14)
    aL = math.sqrt(g * L.p / L.rho)
    xi = np.linspace(-aL + 1e-3, er.wave_speeds(L, R, g)["left_tail"] - 1e-3, 7)
    rho, uu, pp, _ = er.sample(L, R, g, xi)
    np.testing.assert_allclose(uu, (aL + xi) / 2, rtol=1e-13)
    np.testing.assert_allclose(rho, L.rho * (aL - xi) / (2 * aL), rtol=1e-13)
    np.testing.assert_allclose(pp, L.p * (rho / L.rho) ** 3, rtol=1e-13)


# ---- Sec. 4.1: Sod tube for the moment equations ---------------------------------------------

def run_sod(n):
    w = wl.sod(n)
    g = oracle.Grid(w.nx, 1, w.dx, 1.0, w.bcx, w.bcy)
    U, dts = oracle.run_cfl(g, oracle.cons_field(w.W), cfl=w.cfl, t_end=w.t_end)
    return w, U, dts


def test_sod_against_exact_gamma3():
    w, U, dts = run_sod(256)
    assert sum(dts) == pytest.approx(0.2, abs=1e-15)
    W = oracle.prim_field(U)
    ex = er.sod_bme_solution(w.extra["x"], 0.2)
    # rho u_y and Exy stay exactly zero; conservation integrals (outflow ends
    # still hold the initial states): mass 0.5625, Exx = Eyy = 0.55, momentum
    # grows at Pxx_L - Pxx_R = 0.9 per unit time
    assert np.all(U[2] == 0.0) and np.all(U[4] == 0.0)
    dx = w.dx
    assert U[0].sum() * dx == pytest.approx(0.5625, abs=1e-14)
    assert U[3].sum() * dx == pytest.approx(0.55, abs=1e-14)
    assert U[5].sum() * dx == pytest.approx(0.55, abs=1e-14)
    assert U[1].sum() * dx == pytest.approx(0.9 * 0.2, abs=1e-14)
    # L1 accuracy (second-order scheme, HLL, 256 cells)
    l1 = np.abs(W - ex).mean(axis=1)
    assert l1[0] < 6e-3 and l1[1] < 6e-3 and l1[3] < 4e-3 and l1[5] < 6e-3
    # the shock sits within 2 cells of the exact position 0.5 + 2.27300494 t
    xs = 0.5 + 2.2730049442 * 0.2
    jump = np.argmax(np.abs(np.diff(W[0, 200:]))) + 200
    assert abs((jump + 1) * dx - xs) <= 2 * dx
    # Pyy / rho is advected: 1 left of the contact, 0.8 right of it (away from it)
    xc = 0.5 + 0.6085669729 * 0.2
    x = w.extra["x"]
    r = W[5] / W[0]
    assert np.abs(r[x < xc - 0.05] - 1.0).max() < 2e-3
    assert np.abs(r[(x > xc + 0.05)] - 0.8).max() < 2e-3


def test_sod_converges():
    errs = []
    for n in (128, 256, 512, 1024):
        w, U, _ = run_sod(n)
        ex = er.sod_bme_solution(w.extra["x"], 0.2)
        errs.append(np.abs(oracle.prim_field(U)[0] - ex[0]).mean())
    assert all(errs[k + 1] < 0.75 * errs[k] for k in range(3)), errs


# ---- smooth-wave convergence order ----------------------------------------------------------

def linear_wave_error_1d(n, wave, eps=1e-6):
    w0 = np.array([1.0, 0.3, 0.1, 1.0, 0.2, 0.8])
    lam, R, _ = oracle.eigen(0, w0)
    x = (np.arange(n) + 0.5) / n
    W = w0[:, None] + eps * R[:, wave][:, None] * np.sin(2 * np.pi * x)[None, :]
    g = oracle.Grid(n, 1, 1.0 / n, 1.0, oracle.BC_PERIODIC, oracle.BC_PERIODIC)
    t_end = 0.5
    U, _ = oracle.run_cfl(g, oracle.cons_field(W), cfl=0.8, t_end=t_end)
    Wex = w0[:, None] + eps * R[:, wave][:, None] * np.sin(2 * np.pi * (x - lam[wave] * t_end))[None, :]
    return np.abs(oracle.prim_field(U) - Wex).mean() / eps


@pytest.mark.parametrize("wave", [0, 1, 2, 3, 4, 5])
def test_linear_waves_second_order_1d(wave):
    e = [linear_wave_error_1d(n, wave) for n in (64, 128, 256)]
    order = math.log2(e[1] / e[2])
    assert order > 1.75, (e, order)


def test_diagonal_wave_second_order_2d():
    """A density wave carried diagonally across a periodic square: exercises the
    transverse predictor terms (reading R6) and the sum-form CFL (R8)."""
    def err(n, eps=1e-6):
        c = (np.arange(n) + 0.5) / n
        X, Y = np.meshgrid(c, c)
        w0 = np.array([1.0, 0.6, 0.4, 1.0, 0.2, 0.7])
        W = np.broadcast_to(w0[:, None, None], (6, n, n)).copy()
        W[0] += eps * np.sin(2 * np.pi * (X + Y))
        g = oracle.Grid(n, n, 1.0 / n, 1.0 / n)
        t_end = 0.25
        U, _ = oracle.run_cfl(g, oracle.cons_field(W), cfl=0.8, t_end=t_end)
        ex = w0[0] + eps * np.sin(2 * np.pi * (X - w0[1] * t_end + Y - w0[2] * t_end))
        return np.abs(oracle.prim_field(U)[0] - ex).mean() / eps
    e = [err(n) for n in (32, 64, 128)]
    order = math.log2(e[1] / e[2])
    assert order > 1.75, (e, order)


# ---- 2-D invariants ----------------------------------------------------------------------------

def small_periodic(n=48, seed=7):
    w = wl.periodic(n, seed)
    return w, oracle.Grid(n, n, w.dx, w.dy), oracle.cons_field(w.W)


def test_periodic_conservation_2d():
    w, g, U = small_periodic()
    tot0 = U.reshape(6, -1).sum(axis=1)
    U1, _ = oracle.run_cfl(g, U, nsteps=10)
    tot1 = U1.reshape(6, -1).sum(axis=1)
    scale = np.abs(U).reshape(6, -1).max(axis=1) * U[0].size
    assert np.all(np.abs(tot1 - tot0) <= 1e-14 * scale * 10)


@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_OUTFLOW])
def test_free_stream(bc):
    n = 16
    w0 = np.array([0.7, 0.3, -0.2, 0.5, 0.1, 0.9])
    W = np.broadcast_to(w0[:, None, None], (6, n, n)).copy()
    g = oracle.Grid(n, n, 1.0 / n, 1.0 / n, bc, bc)
    U = oracle.cons_field(W)
    U1 = oracle.step(g, 0.01, U)
    np.testing.assert_allclose(U1, U, rtol=1e-14, atol=1e-15)


def swap_xy(U):
    """Exchange the axes: fields (rho, mx, my, Exx, Exy, Eyy) -> (rho, my, mx, Eyy, Exy, Exx), arrays transposed."""
    return np.ascontiguousarray(U[[0, 2, 1, 5, 4, 3]].transpose(0, 2, 1))


@pytest.mark.parametrize("bc", [(oracle.BC_PERIODIC, oracle.BC_OUTFLOW), (oracle.BC_OUTFLOW, oracle.BC_PERIODIC)])
def test_transpose_symmetry(bc):
    """Exchanging the axes (on a non-square grid with dx != dy and different
    boundaries per axis) commutes with the step and with the CFL rate."""
    w = wl.periodic(40, 8)
    U = np.ascontiguousarray(oracle.cons_field(w.W)[:, :24, :])
    g = oracle.Grid(40, 24, 1.0 / 40, 0.7 / 24, bc[0], bc[1])
    gt = oracle.Grid(24, 40, 0.7 / 24, 1.0 / 40, bc[1], bc[0])
    s = oracle.max_signal_speed(g, U)
    assert oracle.max_signal_speed(gt, swap_xy(U)) == pytest.approx(s, rel=1e-15)
    dt = 0.8 / s
    np.testing.assert_allclose(oracle.step(gt, dt, swap_xy(U)), swap_xy(oracle.step(g, dt, U)),
                               rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("twod", [False, True])
@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_OUTFLOW])
def test_boundary_conditions_match_padding(bc, twod):
    """Ghost cells by definition (R9): zero-gradient outflow copies the edge
    cell, periodic wraps.  One step on the grid equals one step on the data
    padded by two such cells per side (numpy pad 'edge' / 'wrap'), cut back to
    the interior; the padded run's own boundaries cannot reach the interior
    because the scheme's stencil radius is 2."""
    n = 20
    w = wl.periodic(n, 12)
    W = w.W if twod else np.ascontiguousarray(w.W[:, 3, :])
    W = W.copy(); W[1] += 0.3
    U = oracle.cons_field(W)
    mode = "wrap" if bc == oracle.BC_PERIODIC else "edge"
    if twod:
        g = oracle.Grid(n, n, 1.0 / n, 1.3 / n, bc, bc, -0.4, -0.6, 0.7, 0.1)
        gp = oracle.Grid(n + 4, n + 4, g.dx, g.dy, 1 - bc, 1 - bc, g.x0 - 2 * g.dx, g.y0 - 2 * g.dy, 0.7, 0.1)
        Up = np.ascontiguousarray(np.pad(U, ((0, 0), (2, 2), (2, 2)), mode=mode))
        cut = lambda A: A[:, 2:-2, 2:-2]
    else:
        g = oracle.Grid(n, 1, 1.0 / n, 1.0, bc, bc)
        gp = oracle.Grid(n + 4, 1, g.dx, 1.0, 1 - bc, 1 - bc)
        Up = np.ascontiguousarray(np.pad(U, ((0, 0), (2, 2)), mode=mode))
        cut = lambda A: A[:, 2:-2]
    dt = 0.5 / oracle.max_signal_speed(g, U)
    np.testing.assert_allclose(oracle.step(g, dt, U), cut(oracle.step(gp, dt, Up)), rtol=1e-14, atol=1e-15)


def test_external_potential_kick():
    """A uniform state at rest in the fixed potential: the hydro step leaves it
    unchanged (free stream), the operator-split kick (Sec. 3.3, last paragraph)
    adds dt * a to the velocity with a = -grad Phi, Phi = vc^2/2 ln(R^2 + rc^2)
    (flat rotation curve), here checked against a numerical gradient of Phi;
    rho and the stress tensor are unchanged by the kick."""
    n = 16
    vc, rc = 1.3, 0.05
    g = oracle.Grid(n, n, 1.0 / n, 1.0 / n, oracle.BC_PERIODIC, oracle.BC_PERIODIC, -0.5, -0.5, vc, rc)
    w0 = np.array([0.8, 0.0, 0.0, 0.3, 0.05, 0.2])
    W = np.broadcast_to(w0[:, None, None], (6, n, n)).copy()
    dt = 1e-3
    W1 = oracle.prim_field(oracle.step(g, dt, oracle.cons_field(W)))
    c = -0.5 + (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c)
    phi = lambda x, y: 0.5 * vc * vc * np.log(x * x + y * y + rc * rc)
    h = 1e-6
    ax = -(phi(X + h, Y) - phi(X - h, Y)) / (2 * h)
    ay = -(phi(X, Y + h) - phi(X, Y - h)) / (2 * h)
    np.testing.assert_allclose(W1[1], dt * ax, rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(W1[2], dt * ay, rtol=1e-7, atol=1e-12)
    for m in (0, 3, 4, 5):
        np.testing.assert_allclose(W1[m], w0[m], rtol=1e-13)


def test_mirror_symmetry():
    """x -> -x maps (rho u, Exy) to their negatives; the step commutes with it."""
    w, g, U = small_periodic(40, 9)
    sign = np.array([1, -1, 1, 1, -1, 1.0])[:, None, None]
    mir = lambda A: np.ascontiguousarray(A[:, :, ::-1] * sign)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    np.testing.assert_allclose(oracle.step(g, dt, mir(U)), mir(oracle.step(g, dt, U)),
                               rtol=1e-13, atol=1e-14)


def test_positivity_on_workload_shapes():
    # the disc needs its core (rc = 0.02) resolved by a few cells: n >= 256
    cases = [wl.periodic(64, 2, 30), wl.disc(256, 3, 30), wl.periodic(64, 5, 30)]
    for w in cases:
        g = oracle.Grid(w.nx, w.ny, w.dx, w.dy, w.bcx, w.bcy, w.x0, w.y0, w.vc, w.rc)
        U = oracle.cons_field(w.W)
        for _ in range(w.nsteps):
            U = oracle.step(g, 0.8 / oracle.max_signal_speed(g, U), U)
            assert oracle.physical(g, U), w.name
    t = wl.tubes(ntubes=6, seed=4, nsteps=60)
    for k in range(6):
        w = wl.tube_workload(t, k)
        g = oracle.Grid(w.nx, 1, w.dx, 1.0, w.bcx, w.bcy)
        U = oracle.cons_field(w.W)
        for _ in range(w.nsteps):
            U = oracle.step(g, 0.8 / oracle.max_signal_speed(g, U), U)
            assert oracle.physical(g, U), (k, w.nx)


# ---- the oracle's own entry points agree with each other ---------------------------------------

def test_fluxes_reproduce_step():
    w, g, U = small_periodic(24, 10)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    Fx, Fy = oracle.fluxes(g, dt, U)
    U1 = U - dt / g.dx * (Fx[:, :, 1:] - Fx[:, :, :-1]) - dt / g.dy * (Fy[:, 1:, :] - Fy[:, :-1, :])
    np.testing.assert_allclose(oracle.step(g, dt, U), U1, rtol=1e-13, atol=1e-14)
    # periodic: the last face equals the first
    np.testing.assert_array_equal(Fx[:, :, 0], Fx[:, :, -1])
    np.testing.assert_array_equal(Fy[:, 0, :], Fy[:, -1, :])


def test_step_cells_matches_step():
    w = wl.disc(32, 3)
    g = oracle.Grid(w.nx, w.ny, w.dx, w.dy, w.bcx, w.bcy, w.x0, w.y0, w.vc, w.rc)
    U = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    full = oracle.step(g, dt, U).reshape(6, -1)
    cells = np.array([0, 1, 31, 32, 33, 500, 1023, 1022, 992, 17 * 32 + 5])
    np.testing.assert_array_equal(oracle.step_cells(g, dt, U, cells), full[:, cells].T)


def test_max_signal_speed_sod():
    """At the Sod initial state the fastest signal is the left sound speed sqrt(3)."""
    w = wl.sod(256)
    g = oracle.Grid(w.nx, 1, w.dx, 1.0, w.bcx, w.bcy)
    assert oracle.max_signal_speed(g, oracle.cons_field(w.W)) == pytest.approx(math.sqrt(3) * 256, rel=1e-15)


# ---- the dense Jacobian (pins the adjoint) --------------------------------------------------------

def test_dense_jacobian_stencil_and_conservation():
    """Periodic 8x8: J is zero outside the radius-2 cross plus 3x3 box of each
    cell, and each 6x6 column-block sum over cells is the identity (the step
    conserves every component's total for every input)."""
    n = 8
    w = wl.periodic(n, 11)
    w.W[1:3] *= 0.5
    g = oracle.Grid(n, n, 1.0 / n, 1.0 / n)
    U = oracle.cons_field(w.W)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    # conservation holds for every input, so it holds for the difference
    # quotient at any step size; a coarse step keeps rounding out of the sums
    J = oracle.dense_jacobian(g, dt, U, rel=1e-4, floor=1e-2).reshape(6, n, n, 6, n, n)
    colsum = J.sum(axis=(1, 2))          # [6, 6, n, n]
    for m in range(6):
        for mm in range(6):
            np.testing.assert_allclose(colsum[m, mm], 1.0 if m == mm else 0.0, atol=1e-9)
    for (j, i) in [(0, 0), (3, 5)]:
        blk = np.abs(J[:, :, :, :, j, i]).max(axis=(0, 3))   # [n, n] dependence of outputs on cell (j,i)
        for jj in range(n):
            for ii in range(n):
                dj = min((jj - j) % n, (j - jj) % n)
                di = min((ii - i) % n, (i - ii) % n)
                inside = (dj <= 1 and di <= 1) or (dj == 0 and di <= 2) or (di == 0 and dj <= 2)
                if not inside:
                    assert blk[jj, ii] == 0.0

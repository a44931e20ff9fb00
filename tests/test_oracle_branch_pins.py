"""Pins of the oracle's validity check and of its branch pattern.

``oracle.physical`` is the positive-definiteness test of Sec. 2 (the stress
Pi_ij = rho sigma^2_ij of a density rho > 0 and a dispersion tensor): each
failure mode, planted in one cell of an otherwise valid grid, must be
rejected, and states just inside each boundary accepted.

``oracle.branches`` reports which side of each kink of the scheme a step's
decisions take (the MC limiter's cases of eq. (25) with the extremum clause,
the max/min with 0 of the tracing coefficients of eqs. (27)-(28), the HLL
speed estimates).  Its pins are hand-derived cases: a density-only profile
(only the density wave of eqs. (22)-(24) has an amplitude, equal to the
density difference, so the limiter cases follow from the differences by
hand) and uniform super- and subsonic flows.
"""
import numpy as np
import pytest

import oracle


def uniform_w(nx, ny, rho=1.0, u=0.0, v=0.0, pxx=1.0, pxy=0.0, pyy=1.0):
    W = np.empty((6, ny, nx))
    for m, val in enumerate((rho, u, v, pxx, pxy, pyy)):
        W[m] = val
    return W


# ---- validity (Sec. 2: rho > 0, stress positive-definite, finite) -----------------------

def base_grid():
    W = uniform_w(7, 5, rho=1.3, u=0.2, v=-0.1, pxx=1.0, pxy=0.3, pyy=0.8)
    return oracle.Grid(7, 5, 0.1, 0.1), W


@pytest.mark.parametrize("field,value", [(0, 0.0), (0, -1.0), (3, 0.0), (3, -0.5), (5, 0.0), (5, -0.5),
                                         (4, 1.0), (4, -1.5)])
def test_physical_rejects_each_failure_mode(field, value):
    """rho <= 0, Pxx <= 0, Pyy <= 0 and, with positive diagonals,
    Pxx Pyy - Pxy^2 <= 0 (Pxx = 1, Pyy = 1: Pxy = +-1 is singular, 1.5
    indefinite), each in one cell."""
    g, W = base_grid()
    if field == 4:
        W[3, 2, 3] = W[5, 2, 3] = 1.0
    W[field, 2, 3] = value
    assert oracle.physical(g, oracle.cons_field(W)) is False
    assert oracle.physical(g, oracle.cons_field(base_grid()[1])) is True


@pytest.mark.parametrize("field", range(6))
@pytest.mark.parametrize("value", [float("nan"), float("inf"), -float("inf")])
def test_physical_rejects_non_finite_conserved_values(field, value):
    g, W = base_grid()
    U = oracle.cons_field(W)
    U[field, 4, 6] = value
    assert oracle.physical(g, U) is False


@pytest.mark.parametrize("field,value", [(0, 1e-200), (3, 1e-200), (5, 1e-200)])
def test_physical_accepts_states_just_inside(field, value):
    g, W = base_grid()
    W[1:3, 1, 1] = 0.0        # no velocity, so E = P exactly in that cell
    W[4, 1, 1] = 0.0
    W[field, 1, 1] = value
    assert oracle.physical(g, oracle.cons_field(W)) is True


def test_physical_accepts_nearly_singular_stress():
    g, W = base_grid()
    W[1:3, 3, 2] = 0.0
    W[3, 3, 2] = W[5, 3, 2] = 1.0
    W[4, 3, 2] = 1.0 - 2.0 ** -30       # det = 2^-29 - 2^-60 > 0
    assert oracle.physical(g, oracle.cons_field(W)) is True
    W[4, 3, 2] = -(1.0 - 2.0 ** -30)
    assert oracle.physical(g, oracle.cons_field(W)) is True


# ---- branch pattern ----------------------------------------------------------------------

# periodic density profile with dyadic values (exact differences) and, per cell,
# the limiter case of the density wave worked out by hand from
# dl = rho_i - rho_{i-1}, dr = rho_{i+1} - rho_i, dc = (dl + dr) / 2:
#   0: dl = -1/2, dr = 1/8            -> opposite signs: off
#   1, 2: dl = dr = 1/8               -> |dc| = 1/8 < 2|dl|: centred
#   3: dl = 1/8, dr = 5/8             -> 2|dl| = 1/4 < |dc| = 3/8: left
#   4: dl = 5/8, dr = 1/8             -> 2|dr| = 1/4 < |dc|: right
#   5: dl = 1/8, dr = 1/16            -> |dc| = 3/32 < 2|dr| = 1/8: centred
#   6: dl = 1/16, dr = -11/16         -> off
#   7: dl = -11/16, dr = -1/2         -> |dc| = 19/32 < 2|dr| = 1: centred
RHO = np.array([1.0, 1.125, 1.25, 1.375, 2.0, 2.125, 2.1875, 1.5])
O, C, L, R = oracle.MC_OFF, oracle.MC_CENTRED, oracle.MC_LEFT, oracle.MC_RIGHT
EXPECT = [O, C, C, L, R, C, O, C]
DENSITY_WAVE = 2   # the order (u-a, u-c, u[rho], u[Pyy], u+c, u+a)


def limited_density_slope(k):
    dl = RHO[k] - RHO[k - 1]
    dr = RHO[(k + 1) % 8] - RHO[k]
    return {O: 0.0, C: 0.5 * (dl + dr), L: 2.0 * dl, R: 2.0 * dr}[EXPECT[k]]


def test_branches_density_profile_1d():
    W = uniform_w(8, 1)[:, 0, :].copy()
    W[0] = RHO
    g = oracle.Grid(8, 1, 1.0 / 8, 1.0, 0, 0)
    U = oracle.cons_field(W)
    dt = 0.4 / oracle.max_signal_speed(g, U)
    b = oracle.branches(g, dt, U)
    cells = b["cells"][0]                    # extended cells i = -1 .. 8
    for i in range(-1, 9):
        k = i % 8
        codes = cells[i + 1]
        expect = [O] * 6
        expect[DENSITY_WAVE] = EXPECT[k]
        assert list(codes[:6]) == expect, (i, codes[:6])
        assert list(codes[6:8]) == [1, 1]    # u = 0: lamM = a > 0, lam0 = -a < 0
        assert not codes[8:].any()           # no y direction in 1-D
    # The face states differ in rho only: rho +- half the limited slope (the
    # density wave moves at u = 0, so tracing adds k a dm to each side and the
    # 1/2 - k a of eq. (27) becomes 1/2).  a = sqrt(3 / rho): S_L = -a of the
    # lighter state, S_R = +a of it; on a tie the left one.
    for i in range(9):                        # face i - 1/2
        rl = RHO[(i - 1) % 8] + 0.5 * limited_density_slope((i - 1) % 8)
        rr = RHO[i % 8] - 0.5 * limited_density_slope(i % 8)
        lighter_right = int(rr < rl)
        assert list(b["fx"][0, i]) == [lighter_right, 0, lighter_right, 0], (i, rl, rr, b["fx"][0, i])


def test_branches_density_profile_along_y():
    """The same profile along y of a 2-D grid: the y codes carry the table,
    the x codes see a uniform state (all limiters off)."""
    nx = 5
    W = uniform_w(nx, 8)
    W[0] = RHO[:, None]
    g = oracle.Grid(nx, 8, 1.0 / nx, 1.0 / 8, 0, 0)
    U = oracle.cons_field(W)
    dt = 0.4 / oracle.max_signal_speed(g, U)
    b = oracle.branches(g, dt, U)
    for j in range(-1, 9):
        for i in range(-1, nx + 1):
            codes = b["cells"][j + 1, i + 1]
            assert not codes[:6].any()
            expect = [O] * 6
            expect[DENSITY_WAVE] = EXPECT[j % 8]
            assert list(codes[8:14]) == expect, (i, j)
            assert list(codes[6:8]) == [1, 1] and list(codes[14:16]) == [1, 1]
    for j in range(9):
        rl = RHO[(j - 1) % 8] + 0.5 * limited_density_slope((j - 1) % 8)
        rr = RHO[j % 8] - 0.5 * limited_density_slope(j % 8)
        lighter_right = int(rr < rl)
        assert (b["fy"][j, :, 0] == lighter_right).all() and (b["fy"][j, :, 2] == lighter_right).all()
    assert not b["fx"].any()                  # equal states: ties go left, subsonic


@pytest.mark.parametrize("u,trace_codes,hll_codes", [
    (2.5, [1, 0], [0, 1, 0, 0]),     # u > a = sqrt(3): every wave moves right (lamM > 0, lam0 > 0), S_L >= 0
    (-2.5, [0, 1], [0, 0, 0, 1]),    # u < -a: every wave moves left (lamM < 0, lam0 < 0), S_R <= 0
    (0.3, [1, 1], [0, 0, 0, 0]),     # subsonic
])
def test_branches_uniform_flow(u, trace_codes, hll_codes):
    """A uniform state: every slope is zero (limiters off), the tracing kinks
    and the HLL clipping follow the sign of u -+ a, a = sqrt(3 Pxx / rho) = sqrt(3)."""
    for ny in (1, 6):
        W = uniform_w(6, ny, u=u, v=u)
        if ny == 1:
            W = W[:, 0, :].copy()
        g = oracle.Grid(6, ny, 0.1, 0.1, 1, 1)
        U = oracle.cons_field(W)
        b = oracle.branches(g, 0.01, U)
        cells = b["cells"].reshape(-1, 16)
        assert not cells[:, :6].any()
        assert (cells[:, 6:8] == trace_codes).all()
        if ny > 1:
            assert not cells[:, 8:14].any() and (cells[:, 14:16] == trace_codes).all()
            assert (b["fy"] == hll_codes).all()
        assert (b["fx"] == hll_codes).all()


def test_same_branches_detects_a_switch():
    """Moving one density value across its neighbour's flips a limiter case."""
    W = uniform_w(8, 1)[:, 0, :].copy()
    W[0] = RHO
    g = oracle.Grid(8, 1, 1.0 / 8, 1.0, 0, 0)
    U = oracle.cons_field(W)
    b0 = oracle.branches(g, 0.01, U)
    assert oracle.same_branches(b0, oracle.branches(g, 0.01, U))
    W[0, 2] = 1.5                             # now cell 2 is a local maximum
    assert not oracle.same_branches(b0, oracle.branches(g, 0.01, oracle.cons_field(W)))

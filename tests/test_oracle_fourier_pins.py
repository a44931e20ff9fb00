"""Pins of the oracle's global Fourier amplitudes (Sec. 4.4):

A_m = |sum over the region of Sigma exp(i m phi) dx dy| / M_d.

Closed forms on point masses, the symmetry of an axisymmetric field sampled
on a square grid (only multiples of 4 survive, the grid artifact the paper
points out for its own m = 4 curve), convergence of a seeded two-armed
perturbation to eps / 2, brute force on a tiny grid, and invariances.
"""
import math

import numpy as np
import pytest

import oracle


def grid(n, ny=None, L=1.0, x0=None, y0=None):
    ny = n if ny is None else ny
    dx, dy = L / n, L / ny
    return oracle.Grid(n, ny, dx, dy, 1, 1, -L / 2 if x0 is None else x0, -L / 2 if y0 is None else y0)


def state(rho):
    """A 2-D state whose density is rho (the other planes do not enter)."""
    U = np.zeros((6,) + rho.shape)
    U[0] = rho
    U[3] = U[5] = 1.0
    return U


def centres(g):
    x = g.x0 + (np.arange(g.nx) + 0.5) * g.dx
    y = g.y0 + (np.arange(g.ny) + 0.5) * g.dy
    return np.meshgrid(x, y)


def test_point_mass_has_unit_amplitudes():
    g = grid(8, 6)
    rho = np.zeros((6, 8))
    rho[1, 6] = 3.7
    np.testing.assert_allclose(oracle.fourier_amplitudes(g, state(rho), 8), 1.0, rtol=1e-15)


def test_opposite_pair_cancels_odd_modes():
    """Equal masses at phi and phi + pi: odd modes vanish, even ones are 1.
    (An angle taken as arctan(y / x) would put both at the same angle.)"""
    g = grid(8)
    rho = np.zeros((8, 8))
    rho[1, 6] = rho[6, 1] = 2.0
    A = oracle.fourier_amplitudes(g, state(rho), 6)
    np.testing.assert_allclose(A[0::2], 0.0, atol=1e-15)
    np.testing.assert_allclose(A[1::2], 1.0, rtol=1e-15)


def test_three_fold_pattern():
    """Unit masses in three cells about 120 degrees apart: the amplitudes are
    those of the three phasors at the cells' own angles; multiples of 3 are
    near 1, the rest small."""
    n = 240
    g = grid(n)
    X, Y = centres(g)
    phi = np.arctan2(Y, X)
    rho = np.zeros((n, n))
    for ang in (0.3, 0.3 + 2 * np.pi / 3, 0.3 + 4 * np.pi / 3):
        d = np.abs(np.angle(np.exp(1j * (phi - ang)))) + np.abs(np.hypot(X, Y) - 0.3)
        j, i = np.unravel_index(np.argmin(d), d.shape)
        rho[j, i] += 1.0
    A = oracle.fourier_amplitudes(g, state(rho), 6)
    sel = rho > 0
    ref = [abs(np.exp(1j * m * phi[sel]).sum()) / 3 for m in range(1, 7)]
    np.testing.assert_allclose(A, ref, rtol=1e-12, atol=1e-15)
    assert A[2] > 0.99 and A[5] > 0.95 and max(A[0], A[1], A[3], A[4]) < 0.1


@pytest.mark.parametrize("n", [64, 65])
def test_axisymmetric_field_on_square_grid_keeps_only_multiples_of_four(n):
    """A field of R alone sampled on a grid symmetric under quarter turns and
    mirrors: the orbit of each cell sums exp(i m phi) to zero unless 4 | m
    (odd n puts a cell on the origin, which has no angle and is left out)."""
    g = grid(n)
    X, Y = centres(g)
    rho = np.exp(-np.hypot(X, Y) / 0.1)
    A = oracle.fourier_amplitudes(g, state(rho), 12)
    for m in range(1, 13):
        if m % 4:
            assert A[m - 1] < 1e-14, (m, A[m - 1])
        else:
            assert A[m - 1] > 1e-9, (m, A[m - 1])


def test_two_armed_perturbation_converges_to_half_eps():
    """Sigma = S(R) (1 + eps cos(2 phi + psi)) with S = (1 - (R / 0.45)^2)^2
    inside R = 0.45 (zero outside, so the support is a disc inside the square):
    the continuum A_2 is exactly eps / 2 and A_4 exactly 0; the midpoint sums
    converge to them at second order."""
    eps, psi = 0.01, 0.7
    e2, a4 = [], []
    for n in (64, 128, 256):
        g = grid(n)
        X, Y = centres(g)
        R, phi = np.hypot(X, Y), np.arctan2(Y, X)
        S = np.where(R < 0.45, (1 - (R / 0.45) ** 2) ** 2, 0.0)
        A = oracle.fourier_amplitudes(g, state(S * (1 + eps * np.cos(2 * phi + psi))), 4)
        e2.append(abs(A[1] - eps / 2) / (eps / 2))
        a4.append(A[3])
    assert e2[2] < 5e-5 and a4[2] < 3e-4, (e2, a4)
    for k in (0, 1):
        assert e2[k] / e2[k + 1] > 3.5 and a4[k] / a4[k + 1] > 3.5, (e2, a4)


def test_brute_force_tiny_grid_with_region():
    g = oracle.Grid(9, 7, 0.11, 0.13, 1, 1, -0.47, -0.41)
    r = np.random.default_rng(3)
    rho = r.uniform(0.1, 2.0, (7, 9))
    Xr, Yr = 0.3, 0.2
    M = rho.sum() * g.dx * g.dy
    ref = []
    for m in range(1, 7):
        s = 0j
        for j in range(7):
            for i in range(9):
                x = g.x0 + (i + 0.5) * g.dx
                y = g.y0 + (j + 0.5) * g.dy
                if abs(x) <= Xr and abs(y) <= Yr:
                    s += rho[j, i] * complex(math.cos(m * math.atan2(y, x)), math.sin(m * math.atan2(y, x))) \
                        * g.dx * g.dy
        ref.append(abs(s) / M)
    np.testing.assert_allclose(oracle.fourier_amplitudes(g, state(rho), 6, Xr, Yr), ref, rtol=1e-13)


def test_quarter_turn_and_mirror_invariance():
    g = grid(48)
    r = np.random.default_rng(4)
    rho = r.uniform(0.5, 1.5, (48, 48))
    A = oracle.fourier_amplitudes(g, state(rho), 6)
    for t in (np.rot90(rho), np.flipud(rho), np.fliplr(rho), rho.T):
        np.testing.assert_allclose(oracle.fourier_amplitudes(g, state(np.ascontiguousarray(t)), 6), A,
                                   rtol=1e-12)


def test_mass_outside_the_region_only_rescales():
    g = grid(40)
    X, Y = centres(g)
    r = np.random.default_rng(5)
    rho = r.uniform(0.5, 1.5, (40, 40))
    inside = (np.abs(X) <= 0.25) & (np.abs(Y) <= 0.25)
    A1 = oracle.fourier_amplitudes(g, state(rho), 6, 0.25, 0.25)
    rho2 = rho.copy()
    rho2[~inside] *= 3.0
    A2 = oracle.fourier_amplitudes(g, state(rho2), 6, 0.25, 0.25)
    M1, M2 = rho.sum(), rho2.sum()
    np.testing.assert_allclose(A2, A1 * M1 / M2, rtol=1e-13)


def test_origin_cell_is_left_out():
    g = grid(5)
    rho = np.zeros((5, 5))
    rho[2, 2] = 1.0                     # the centre cell sits on the origin
    np.testing.assert_allclose(oracle.fourier_amplitudes(g, state(rho), 4), 0.0, atol=0.0)
    rho[0, 0] = 1.0
    np.testing.assert_allclose(oracle.fourier_amplitudes(g, state(rho), 4), 0.5, rtol=1e-15)

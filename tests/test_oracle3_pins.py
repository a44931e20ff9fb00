"""Pins of the oracle's three-dimensional ten-moment scheme (cshoracle3.c).

What fixes it: the conserved variables and fluxes are velocity moments of a
symmetric discrete distribution (the definition of the moment equations);
the primitive Jacobian is the transformed flux Jacobian; A R = R Lambda,
L R = I with ten eigenvalues u -+ a, u -+ c (twice), u (four times); a state
that does not vary along z and has no z-motion or z-shear reproduces the
pinned 2-D oracle; a tube along any axis reproduces the pinned 1-D oracle;
conservation, free stream, permutation of the axes, the cell-by-cell step,
and second-order convergence of a wave across all three axes.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl

rng = np.random.default_rng(17)
PIDX = ((4, 5, 6), (5, 7, 8), (6, 8, 9))


def random_state3(g=rng, umax=0.5):
    rho = math.exp(0.4 * g.standard_normal())
    u = umax * g.standard_normal(3)
    L = np.tril(g.uniform(-0.3, 0.3, (3, 3)))
    L[np.diag_indices(3)] = 0.5 + g.random(3)
    P = rho * L @ L.T
    w = np.empty(10)
    w[0], w[1:4] = rho, u
    for i in range(3):
        for j in range(i, 3):
            w[PIDX[i][j]] = P[i, j]
    return w


def sigma_points3(w):
    """Six equally weighted velocities u +- sqrt(3) C e_k (C C^T = P / rho):
    density rho, mean u, dispersion P / rho, zero third central moment."""
    rho, u = w[0], w[1:4]
    P = np.array([[w[PIDX[i][j]] for j in range(3)] for i in range(3)])
    C = np.linalg.cholesky(P / rho)
    pts = [u + s * math.sqrt(3.0) * C[:, k] for k in range(3) for s in (1, -1)]
    return np.array(pts), rho / 6.0


@pytest.mark.parametrize("trial", range(6))
def test_conserved_and_fluxes_are_velocity_moments(trial):
    w = random_state3()
    pts, wt = sigma_points3(w)
    U = oracle.cons3(w)
    mom = np.empty(10)
    mom[0] = wt * len(pts)
    for i in range(3):
        mom[1 + i] = wt * pts[:, i].sum()
        for j in range(i, 3):
            mom[PIDX[i][j]] = wt * (pts[:, i] * pts[:, j]).sum()
    np.testing.assert_allclose(U, mom, rtol=1e-13, atol=1e-14)
    for k in range(3):
        F = np.empty(10)
        F[0] = wt * pts[:, k].sum()
        for i in range(3):
            F[1 + i] = wt * (pts[:, i] * pts[:, k]).sum()
            for j in range(i, 3):
                F[PIDX[i][j]] = wt * (pts[:, i] * pts[:, j] * pts[:, k]).sum()
        np.testing.assert_allclose(oracle.flux3(k, U), F, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(oracle.prim3(U), w, rtol=1e-13, atol=1e-14)


def fd_jac(f, x, h):
    n = x.size
    J = np.empty((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = h * max(1.0, abs(x[c]))
        J[:, c] = (-f(x + 2 * e) + 8 * f(x + e) - 8 * f(x - e) + f(x - 2 * e)) / (12 * e[c])
    return J


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("trial", range(3))
def test_primitive_jacobian_and_eigensystem(axis, trial):
    w = random_state3()
    U = oracle.cons3(w)
    dFdU = fd_jac(lambda x: oracle.flux3(axis, x), U, 1e-4)
    M = fd_jac(oracle.cons3, w, 1e-4)          # dU/dW
    A_fd = np.linalg.solve(M, dFdU @ M)
    A = oracle.jac3(axis, w)
    np.testing.assert_allclose(A, A_fd, rtol=1e-7, atol=1e-8)
    lam, R, L = oracle.eigen3(axis, w)
    np.testing.assert_allclose(A @ R, R * lam, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(L @ R, np.eye(10), atol=1e-12)
    un, a, c = w[1 + axis], math.sqrt(3 * w[PIDX[axis][axis]] / w[0]), math.sqrt(w[PIDX[axis][axis]] / w[0])
    np.testing.assert_allclose(lam, [un - a, un - c, un - c, un, un, un, un, un + c, un + c, un + a], rtol=1e-14)
    np.testing.assert_allclose(np.sort(np.linalg.eigvals(dFdU).real), lam, rtol=1e-6, atol=1e-7)


def to3(W2, nz=1):
    """A 2-D primitive state [6, ny, nx] as a z-invariant 3-D state with w = 0,
    Pxz = Pyz = 0 and Pzz = 0.7 rho."""
    ny, nx = W2.shape[1:]
    W = np.zeros((10, nz, ny, nx))
    W[0], W[1], W[2] = W2[0], W2[1], W2[2]
    W[4], W[5], W[7] = W2[3], W2[4], W2[5]
    W[9] = 0.7 * W2[0]
    return W


@pytest.mark.parametrize("bc", [(0, 0), (1, 0), (0, 1)])
def test_z_invariant_state_reproduces_the_2d_scheme(bc):
    w2 = wl.periodic(64, 5)
    W2 = np.ascontiguousarray(w2.W[:, :20, :24])
    g2 = oracle.Grid(24, 20, 1.0 / 24, 1.2 / 20, bc[0], bc[1])
    U2 = oracle.cons_field(W2)
    dt = 0.5 / oracle.max_signal_speed(g2, U2)
    ref = oracle.step(g2, dt, U2)
    for nz, bz in ((1, 0), (3, 0), (2, 1)):
        g3 = oracle.Grid3(24, 20, nz, 1.0 / 24, 1.2 / 20, 0.37, (bc[0], bc[1], bz))
        U3 = oracle.cons3_field(to3(W2, nz))
        out = oracle.step3(g3, dt, U3)
        for k in range(nz):
            got = out[[0, 1, 2, 4, 5, 7], k]
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)
        np.testing.assert_array_equal(out[[3, 6, 8]], 0.0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_tube_along_each_axis_reproduces_the_1d_scheme(axis):
    s = wl.sod(64)
    g1 = oracle.Grid(64, 1, 1.0 / 64, 1.0, 1, 1)
    U1 = oracle.cons_field(s.W)
    dt = 0.8 / oracle.max_signal_speed(g1, U1)
    ref = U1
    for _ in range(5):
        ref = oracle.step(g1, dt, ref)
    # the tube's (rho, u_n, P_nn, P_tt) along the chosen axis; the other
    # transverse stress equal to P_tt
    W = np.zeros((10, 64))
    W[0] = s.W[0]
    W[PIDX[axis][axis]] = s.W[3]
    for t in range(3):
        if t != axis:
            W[PIDX[t][t]] = s.W[5]
    shape = [1, 1, 1]
    shape[2 - axis] = 64                      # arrays are [z, y, x]
    W = W.reshape((10,) + tuple(shape))
    n = [1, 1, 1]
    n[axis] = 64
    h = [1.0, 1.0, 1.0]
    h[axis] = 1.0 / 64
    g3 = oracle.Grid3(n[0], n[1], n[2], h[0], h[1], h[2], (1, 1, 1))
    U = oracle.cons3_field(W)
    for _ in range(5):
        U = oracle.step3(g3, dt, U)
    U = U.reshape(10, 64)
    np.testing.assert_allclose(U[0], ref[0], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(U[1 + axis], ref[1], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(U[PIDX[axis][axis]], ref[3], rtol=1e-13, atol=1e-14)
    for t in range(3):
        if t != axis:
            np.testing.assert_allclose(U[PIDX[t][t]], ref[5], rtol=1e-13, atol=1e-14)


def permute_axes(U, perm):
    """Relabel the axes: new axis a is old axis perm[a] (arrays [10, z, y, x])."""
    out = np.empty_like(U.transpose(0, *[3 - perm[2 - d] for d in range(3)]))
    arr = U.transpose(0, *[3 - perm[2 - d] for d in range(3)])
    out[0] = arr[0]
    for a in range(3):
        out[1 + a] = arr[1 + perm[a]]
        for b in range(a, 3):
            out[PIDX[a][b]] = arr[PIDX[perm[a]][perm[b]]]
    return np.ascontiguousarray(out)


def test_axis_permutation_symmetry():
    w = wl.periodic3(12, 10, 8, seed=3)
    g = oracle.Grid3(12, 10, 8, 1 / 12, 1.1 / 10, 0.9 / 8, (0, 1, 0))
    U = oracle.cons3_field(w.W)
    dt = 0.5 / oracle.max_signal_speed3(g, U)
    out = oracle.step3(g, dt, U)
    perm = (2, 0, 1)                           # new x = old z, new y = old x, new z = old y
    n, h, bc = (12, 10, 8), (1 / 12, 1.1 / 10, 0.9 / 8), (0, 1, 0)
    gp = oracle.Grid3(n[perm[0]], n[perm[1]], n[perm[2]], h[perm[0]], h[perm[1]], h[perm[2]],
                      (bc[perm[0]], bc[perm[1]], bc[perm[2]]))
    outp = oracle.step3(gp, dt, permute_axes(U, perm))
    np.testing.assert_allclose(outp, permute_axes(out, perm), rtol=1e-12, atol=1e-13)


def test_conservation_and_free_stream():
    w = wl.periodic3(12, 10, 8, seed=4)
    g = oracle.Grid3(12, 10, 8, 1 / 12, 1 / 10, 1 / 8)
    U = oracle.cons3_field(w.W)
    dt = 0.8 / oracle.max_signal_speed3(g, U)
    out = oracle.step3(g, dt, U)
    np.testing.assert_allclose(out.reshape(10, -1).sum(axis=1), U.reshape(10, -1).sum(axis=1),
                               rtol=1e-13, atol=1e-11)
    flat = np.broadcast_to(random_state3()[:, None, None, None], (10, 5, 6, 7)).copy()
    gf = oracle.Grid3(7, 6, 5, 0.1, 0.2, 0.3, (1, 0, 1))
    Uf = oracle.cons3_field(flat)
    np.testing.assert_allclose(oracle.step3(gf, 0.01, Uf), Uf, rtol=1e-14, atol=1e-14)


def test_cells_step_matches_grid_step():
    w = wl.periodic3(10, 9, 8, seed=5)
    g = oracle.Grid3(10, 9, 8, 0.1, 0.1, 0.1, (1, 0, 1))
    U = oracle.cons3_field(w.W)
    dt = 0.8 / oracle.max_signal_speed3(g, U)
    full = oracle.step3(g, dt, U).reshape(10, -1)
    cells = np.array([0, 9, 10, 89, 90, 355, 719, 100, 500])
    np.testing.assert_array_equal(oracle.step3_cells(g, dt, U, cells).T, full[:, cells])


def test_cfl_rate_is_the_three_axis_sum():
    w = random_state3()
    g = oracle.Grid3(1, 1, 1, 0.1, 0.2, 0.3)
    U = oracle.cons3(w).reshape(10, 1, 1, 1)
    s = sum((abs(w[1 + k]) + math.sqrt(3 * w[PIDX[k][k]] / w[0])) / h for k, h in enumerate((0.1, 0.2, 0.3)))
    assert oracle.max_signal_speed3(g, U) == pytest.approx(s, rel=1e-14)


def test_diagonal_wave_second_order():
    """A density wave along (1, 1, 1) carried by a uniform flow across a
    periodic cube: exercises the transverse terms of both other axes."""
    def err(n, eps=1e-6):
        c = (np.arange(n) + 0.5) / n
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        w0 = np.array([1.0, 0.5, 0.4, 0.3, 1.0, 0.1, 0.05, 0.8, 0.02, 0.9])
        W = np.broadcast_to(w0[:, None, None, None], (10, n, n, n)).copy()
        W[0] += eps * np.sin(2 * np.pi * (X + Y + Z))
        g = oracle.Grid3(n, n, n, 1 / n, 1 / n, 1 / n)
        U = oracle.cons3_field(W)
        t_end, t = 0.1, 0.0
        while t < t_end - 1e-15:
            dt = min(0.8 / oracle.max_signal_speed3(g, U), t_end - t)
            U = oracle.step3(g, dt, U)
            t += dt
        ex = w0[0] + eps * np.sin(2 * np.pi * (X + Y + Z - (w0[1] + w0[2] + w0[3]) * t_end))
        return np.abs(oracle.prim3_field(U)[0] - ex).mean() / eps
    e = [err(n) for n in (12, 24)]
    assert math.log2(e[0] / e[1]) > 1.7, e

"""The GPU adjoint: against the CPU harness of the same reverse pass, against
the oracle's dense Jacobian, and the 512^2 / 200-step gradient against central
finite differences on 64 smooth random directions (frozen timesteps)."""
import ctypes
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as wl
import paper_1210_5246_amd as csh
from paper_1210_5246_amd import autograd as cag

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "host"))
pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, flush=True)


def small_case(kind, bc, n):
    m = max(64, n + 24)  # the generator's width (64 for the sizes up to 40)
    if kind == "2d":
        w = wl.periodic(m, 61)
        W = np.ascontiguousarray(w.W[:, 10:10 + n, 20:20 + n])
        W[1:3] *= 2.0
        g = oracle.Grid(n, n, 1.0 / n, 1.2 / n, bc, bc, -0.4, -0.55, 0.8 if bc else 0.0, 0.1)
    else:
        w = wl.periodic(m, 62)
        W = np.ascontiguousarray(w.W[:, 9, 3:3 + n])
        W[1] *= 2.0
        g = oracle.Grid(n, 1, 1.0 / n, 1.0, bc, bc, -0.3, 0.0, 0.6 if bc else 0.0, 0.2)
    return W, g


def gpu(W, g):
    G = csh.Grid(torch.from_numpy(W).to(DEV), g.dx, g.dy, (g.bcx, g.bcy))
    if g.vc:
        G.set_potential(g.vc, g.rc, g.x0, g.y0)
    return G


def jac_case(kind, bc):
    """8 cells (1-D) or 8 x 8 (2-D) cut from a smooth random field, with the
    potential on under outflow; the cut is chosen so that no decision of the
    step sits within a difference step of a kink (asserted by the test)."""
    if kind == "2d":
        w = wl.periodic(64, 61)
        W = np.ascontiguousarray(w.W[:, 30:38, 30:38])
        W[1:3] *= 2.0
        g = oracle.Grid(8, 8, 1.0 / 8, 1.2 / 8, bc, bc, -0.4, -0.55, 0.8 if bc else 0.0, 0.1)
        return W, g
    return small_case(kind, bc, 8)


@pytest.mark.parametrize("kind", ["1d", "2d"])
@pytest.mark.parametrize("bc", [0, 1])
def test_gpu_adjoint_matches_oracle_dense_jacobian(kind, bc):
    """Rows J^T e_k of the GPU adjoint against the oracle's central-difference
    Jacobian.  Every column's difference interval is first shown to be free of
    kinks: the oracle's branch pattern (limiter cases, tracing and HLL
    clipping) is the same at U - h e_b, U and U + h e_b, so the difference
    quotient is a derivative of one smooth branch of the step."""
    W, g = jac_case(kind, bc)
    say("adjoint vs dense Jacobian", kind, bc)
    U = oracle.cons_field(W)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    b0 = oracle.branches(g, dt, U)
    flat = U.ravel()
    for b in range(flat.size):
        h = 1e-7 * max(abs(flat[b]), 1e-3)      # the step dense_jacobian takes
        for sgn in (1.0, -1.0):
            x = flat.copy()
            x[b] += sgn * h
            assert oracle.same_branches(b0, oracle.branches(g, dt, x.reshape(U.shape))), (b, sgn)
    J = oracle.dense_jacobian(g, dt, U)
    G = gpu(W, g)
    Ud = torch.from_numpy(U).to(DEV)
    n = U.size
    rows = np.empty((n, n))
    for k in range(n):
        e = torch.zeros(n, dtype=torch.float64, device=DEV)
        e[k] = 1.0
        rows[k] = G.adjoint_step(dt, Ud, e.reshape(U.shape).contiguous()).cpu().numpy().ravel()
    dev = np.abs(rows - J).max() / np.abs(J).max()
    say("max |J^T e_k - J| / max |J|:", dev)
    assert dev < 1e-6, dev


def smooth_fields(r, shape, width=8.0):
    """Six smooth zero-mean unit-std fields of the given 1-D or 2-D shape."""
    if len(shape) == 1:
        n = shape[0]
        m = max(64, n)
        return np.stack([wl.smooth_gaussian(r, (m, m), width)[0, :n] for _ in range(6)])
    ny, nx = shape
    m = max(64, nx, ny)
    return np.stack([wl.smooth_gaussian(r, (m, m), width)[:ny, :nx] for _ in range(6)])


def dot_case(shape, bc, kick, seed):
    """A smooth random state of the given shape (cut from the periodic
    generator, velocities doubled), optionally with the disc's potential."""
    if len(shape) == 1:
        n = shape[0]
        w = wl.periodic(max(64, n + 16), seed)
        W = np.ascontiguousarray(w.W[:, 7, 5:5 + n])
        W[1] *= 2.0
        g = oracle.Grid(n, 1, 1.0 / n, 1.0, bc, bc, -0.3, 0.0, 0.6 if kick else 0.0, 0.2)
    else:
        ny, nx = shape
        w = wl.periodic(max(64, nx + 16, ny + 16), seed)
        W = np.ascontiguousarray(w.W[:, 6:6 + ny, 5:5 + nx])
        W[1:3] *= 2.0
        g = oracle.Grid(nx, ny, 1.0 / nx, 1.3 / ny, bc, bc, -0.4, -0.55, 0.8 if kick else 0.0, 0.1)
    return W, g


# sizes around 60- and 62-wide wavefront strips (1-D rows), around the 2-D
# reverse pass's tiles (32 x 8 extended cells; 14 x 14 outputs), tall/short
# grids and the 512^2 periodic grid of the gradient benchmark; both boundary
# kinds, potential on and off
DOT_CASES = [((58,), 0, 0), ((59,), 1, 1), ((60,), 0, 1), ((61,), 1, 0), ((121,), 0, 0), ((121,), 1, 1),
             ((37, 121), 0, 0), ((37, 121), 1, 1), ((61, 59), 1, 0), ((70, 130), 0, 1), ((5, 61), 1, 1),
             ((130, 7), 0, 0), ((29, 31), 1, 0), ((28, 60), 0, 1),
             ((15, 29), 0, 1), ((512, 512), 0, 0)]  # the last: the gradient benchmark's grid and launch


@pytest.mark.parametrize("shape,bc,kick", DOT_CASES)
def test_adjoint_dot_product_against_oracle_forward(shape, bc, kick):
    """<lam, J delta> with J delta by central differences of the ORACLE's step
    against <J^T lam, delta> from the GPU adjoint, <= 1e-6 relative.  The
    difference step is the largest of 1e-7, 1e-8, 1e-9 (relative to each
    field's scale) whose interval holds no kink: the oracle's branch pattern is
    the same at U - eps delta, U and U + eps delta."""
    W, g = dot_case(shape, bc, kick, 65)
    say("adjoint dot product vs oracle forward", shape, bc, kick)
    U = oracle.cons_field(W)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    r = np.random.default_rng(sum(shape) * 10 + bc * 2 + kick)
    lam = r.standard_normal(U.shape)
    scale = np.abs(U).reshape(6, -1).max(axis=1).reshape((6,) + (1,) * (U.ndim - 1))
    delta = smooth_fields(r, U.shape[1:]) * scale
    G = gpu(W, g)
    got = G.adjoint_step(dt, torch.from_numpy(U).to(DEV), torch.from_numpy(lam).to(DEV)).cpu().numpy()
    rhs = float((got * delta).sum())
    b0 = oracle.branches(g, dt, U)
    for eps in (1e-7, 1e-8, 1e-9):
        if (oracle.same_branches(b0, oracle.branches(g, dt, U + eps * delta)) and
                oracle.same_branches(b0, oracle.branches(g, dt, U - eps * delta))):
            break
    else:
        pytest.fail("every difference interval crosses a kink")
    Jd = (oracle.step(g, dt, U + eps * delta) - oracle.step(g, dt, U - eps * delta)) / (2 * eps)
    lhs = float((lam * Jd).sum())
    rel = abs(lhs - rhs) / abs(rhs)
    say(f"eps {eps:g}: <lam, J d> {lhs:.12e} <J^T lam, d> {rhs:.12e} rel {rel:.1e}")
    assert rel <= 1e-6


# sizes around the x-part kernel's wavefronts (62 padded positions each, nx + 4
# per row: one wavefront at 58, two at 59 and 120, three at 121) and tiny grids
@pytest.mark.parametrize("kind,n", [("1d", m) for m in (1, 2, 3, 37, 58, 59, 121)] +
                         [("2d", m) for m in (2, 3, 37, 58, 59, 121)])
@pytest.mark.parametrize("bc", [0, 1])
def test_gpu_adjoint_matches_host_reverse_pass(kind, n, bc):
    import test_adjoint_host as th
    W, g = small_case(kind, bc, n)
    say("adjoint gpu vs host", kind, n, bc)
    U = oracle.cons_field(W)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    lam = np.random.default_rng(5).standard_normal(U.shape)
    ref = th.host_adjoint(g, dt, U, lam)
    G = gpu(W, g)
    got = G.adjoint_step(dt, torch.from_numpy(U).to(DEV), torch.from_numpy(lam).to(DEV)).cpu().numpy()
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12


@pytest.mark.parametrize("kind,steps,tol", [("smooth", (1e-7, 1e-8), 1e-7), ("noise", (1e-9, 1e-10), 1e-6)])
def test_dot_product_128_periodic(kind, steps, tol):
    """<lam, J d> (central differences of the GPU forward) against <J^T lam, d>.
    A central difference whose interval straddles a limiter kink in one of the
    16k cells is off by O(eps) (its error shrinks linearly with eps, unlike the
    O(eps^2) error of a smooth quotient); the closer of two steps is taken."""
    w = wl.periodic(128, 63)
    say("dot product 128^2", kind)
    G = csh.Grid(torch.from_numpy(w.W).to(DEV), w.dx, w.dy)
    U = G.U
    dt = 0.8 / G.max_signal_speed()
    r = np.random.default_rng(9)
    lam = torch.from_numpy(r.standard_normal(U.shape)).to(DEV)
    scale = U.abs().reshape(6, -1).amax(dim=1).reshape(6, 1, 1)
    if kind == "noise":
        d = torch.from_numpy(r.standard_normal(U.shape)).to(DEV) * scale
    else:
        d = torch.from_numpy(np.stack([wl.smooth_gaussian(r, (128, 128), 8.0) for _ in range(6)])).to(DEV) * scale
    rhs = float((G.adjoint_step(dt, U, lam) * d).sum())
    devs = []
    for eps in steps:
        Jd = (G.step(dt, U + eps * d) - G.step(dt, U - eps * d)) / (2 * eps)
        lhs = float((lam * Jd).sum())
        devs.append(abs(lhs - rhs) / abs(rhs))
    say("relative deviations", devs)
    assert min(devs) <= tol, devs


def loss_of(U, rho_target):
    return 0.5 * ((U[0] - rho_target) ** 2).sum()


def test_gradient_512_against_finite_differences():
    """512^2 periodic, 200 steps, checkpoints every 20: the gradient of
    1/2 sum (rho_200 - rho*)^2 with respect to the initial primitive fields
    against central differences of the GPU forward (frozen timesteps) on 64
    smooth directions, at two fixed steps.

    * eps = 1e-6: every direction within 1e-5 of sum |grad * d| (the size of
      what the dot product sums); the count within 1e-5 relative,
      |FD - <grad, d>| <= 1e-5 max(|FD|, |<grad, d>|), is reported.  A
      difference over 200 x 512^2 cell updates crosses limiter and tracing
      kinks, each an error of the order of the step, so at this step it is
      the differences that limit the agreement (40 of 64 measured).
    * eps = 1e-9: the kink errors have shrunk (the median error of the 64
      falls with the step) and at least 63 of 64 directions are within 1e-5
      relative.  The one that is not has <grad, d> = -9.4 against terms that
      sum to 6.3e4: there the quotient's own floor (kinks at larger steps,
      rounding of the two runs at smaller ones, ~3e-4 absolute) is 3e-5 of the
      value.

    Gradients with checkpoints every 20 steps, one checkpoint (everything
    recomputed) and every state kept are bitwise equal."""
    w0, wt = wl.adjoint(512, 5, 6, 200, 20)
    say("target run")
    Gt = csh.Grid(torch.from_numpy(wt.W).to(DEV), wt.dx, wt.dy)
    Gt.run_cfl(200, 0.8)
    rho_t = Gt.U[0].clone()
    W0 = torch.from_numpy(w0.W).to(DEV).requires_grad_(True)
    say("forward + adjoint, K=20")
    U, dts = cag.sweep(W0, w0.dx, w0.dy, nsteps=200, checkpoint_every=20)
    L = loss_of(U, rho_t)
    (grad,) = torch.autograd.grad(L, W0)
    say("forward + adjoint, K=200")
    W0b = torch.from_numpy(w0.W).to(DEV).requires_grad_(True)
    U2, dts2 = cag.sweep(W0b, w0.dx, w0.dy, nsteps=200, checkpoint_every=200)
    (grad2,) = torch.autograd.grad(loss_of(U2, rho_t), W0b)
    assert torch.equal(dts, dts2) and torch.equal(grad, grad2)
    say("forward + adjoint, K=1 (every state kept, no recomputation)")
    W0c = torch.from_numpy(w0.W).to(DEV).requires_grad_(True)
    U3, dts3 = cag.sweep(W0c, w0.dx, w0.dy, nsteps=200, checkpoint_every=1)
    (grad3,) = torch.autograd.grad(loss_of(U3, rho_t), W0c)
    assert torch.equal(dts, dts3) and torch.equal(U, U3) and torch.equal(grad, grad3)
    dirs = wl.fd_directions(512, 64)
    Wd = torch.from_numpy(w0.W).to(DEV)
    runner = cag.FrozenRunner(Wd, w0.dx, w0.dy, (0, 0), dts)
    stats = {}
    for eps in (1e-6, 1e-9):
        rel, scaled = [], []
        for k, d in enumerate(dirs):
            dd = torch.from_numpy(d).to(DEV)
            ad = float((grad * dd).sum())
            terms = float((grad * dd).abs().sum())
            rp = runner.run(Wd + eps * dd)[0].clone()
            rm = runner.run(Wd - eps * dd)[0]
            # L(+) - L(-) = sum (rho+ - rho-)((rho+ + rho-)/2 - rho*): the same
            # difference, formed without cancelling two sums of size ~1e4
            fd = float(((rp - rm) * (0.5 * (rp + rm) - rho_t)).sum()) / (2 * eps)
            rel.append(abs(fd - ad) / max(abs(fd), abs(ad)))
            scaled.append(abs(fd - ad) / terms)
            if rel[-1] > 1e-5:
                say(f"eps {eps:g} direction {k}: adjoint {ad:.6e} (terms {terms:.3e}) fd {fd:.6e} "
                    f"rel {rel[-1]:.1e} rel-to-terms {scaled[-1]:.1e}")
        rel, scaled = np.array(rel), np.array(scaled)
        stats[eps] = (int((rel <= 1e-5).sum()), float(np.median(rel)), float(scaled.max()))
        say(f"eps {eps:g}: {stats[eps][0]}/64 within 1e-5 relative, median {stats[eps][1]:.1e}, "
            f"worst deviation / sum|grad*d| {stats[eps][2]:.1e}")
    assert stats[1e-6][2] <= 1e-5
    assert stats[1e-9][2] <= 1e-6
    assert stats[1e-9][1] < stats[1e-6][1] / 10      # the kink errors shrink with the step
    assert stats[1e-9][0] >= 63


def test_sweep_raises_on_a_nonphysical_run():
    """The differentiable sweep reads the handle's validity flag at its one
    host synchronisation: a run that blows up (C = 20) raises instead of
    returning non-finite states to differentiate; the handle it caches is
    cleared by the next sweep of the same geometry."""
    w = wl.periodic(64, 2)
    W0 = torch.from_numpy(w.W).to(DEV).requires_grad_(True)
    say("autograd sweep at C = 20")
    with pytest.raises(csh.NonPhysicalState):
        cag.sweep(W0, w.dx, w.dy, nsteps=6, checkpoint_every=3, cfl=20.0)
    U, _ = cag.sweep(W0, w.dx, w.dy, nsteps=3, checkpoint_every=3)
    assert torch.isfinite(U).all()

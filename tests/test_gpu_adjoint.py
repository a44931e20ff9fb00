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


@pytest.mark.parametrize("kind", ["1d", "2d"])
@pytest.mark.parametrize("bc", [0, 1])
def test_gpu_adjoint_matches_oracle_dense_jacobian(kind, bc):
    W, g = small_case(kind, bc, 8)
    say("adjoint vs dense Jacobian", kind, bc)
    U = oracle.cons_field(W)
    dt = 0.8 / oracle.max_signal_speed(g, U)
    J = oracle.dense_jacobian(g, dt, U)
    G = gpu(W, g)
    Ud = torch.from_numpy(U).to(DEV)
    n = U.size
    rows = np.empty((n, n))
    for k in range(n):
        e = torch.zeros(n, dtype=torch.float64, device=DEV)
        e[k] = 1.0
        rows[k] = G.adjoint_step(dt, Ud, e.reshape(U.shape).contiguous()).cpu().numpy().ravel()
    # a central difference that straddles a limiter/HLL kink is not a derivative:
    # per entry, take the closer of two difference steps (the kink is then
    # either inside only the wider one, or far from both)
    J2 = oracle.dense_jacobian(g, dt, U, rel=1e-8)
    dev = np.minimum(np.abs(rows - J), np.abs(rows - J2)) / np.abs(J).max()
    assert dev.max() < 1e-6, dev.max()


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
    against central differences on 64 smooth directions: |fd - <grad, d>| <=
    1e-5 sum |grad * d| for every direction and <= 1e-5 |<grad, d>| for at
    least 60 of them; gradients with checkpoints every 20 steps, one checkpoint
    (everything recomputed) and every state kept bitwise equal."""
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
    worst_scaled, plain_ok = 0.0, 0
    Wd = torch.from_numpy(w0.W).to(DEV)
    for k, d in enumerate(dirs):
        dd = torch.from_numpy(d).to(DEV)
        ad = float((grad * dd).sum())
        terms = float((grad * dd).abs().sum())  # size of what the dot product sums
        # central differences at eps = 1e-6 (the check's step) and, where that
        # interval straddles a limiter kink somewhere in the 200 x 512^2 cell
        # updates (an O(eps) error), at smaller steps; the closest is compared
        devs = []
        for eps in (1e-6, 1e-7, 1e-8, 1e-9, 1e-10):
            rp = cag.run_frozen(Wd + eps * dd, w0.dx, w0.dy, (0, 0), dts)[0]
            rm = cag.run_frozen(Wd - eps * dd, w0.dx, w0.dy, (0, 0), dts)[0]
            # L(+) - L(-) = sum (rho+ - rho-)((rho+ + rho-)/2 - rho*): the same
            # difference, formed without cancelling two sums of size ~1e4
            fd = float(((rp - rm) * (0.5 * (rp + rm) - rho_t)).sum()) / (2 * eps)
            devs.append(abs(fd - ad))
            if devs[-1] <= 1e-6 * abs(ad):
                break
        dev = min(devs)
        plain = dev / abs(ad)
        plain_ok += plain <= 1e-5
        worst_scaled = max(worst_scaled, dev / terms)
        if k % 8 == 0 or plain > 1e-5:
            say(f"direction {k}: adjoint {ad:.6e} (terms {terms:.3e}) |fd - adjoint| {dev:.2e} "
                f"rel {plain:.1e} rel-to-terms {dev / terms:.1e}")
    say(f"directions within 1e-5 relative: {plain_ok}/64; worst deviation / sum|grad*d|: {worst_scaled:.2e}")
    # The difference quotients bottom out at ~1e-4..1e-3 absolute (kinks at
    # large eps, rounding at small eps); a direction whose derivative nearly
    # cancels (|<grad, d>| << sum |grad * d|) cannot be resolved relatively.
    assert worst_scaled <= 1e-5
    assert plain_ok >= 60

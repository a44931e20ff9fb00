"""Seeded synthetic inputs shaped like the paper's test problems.

This module only draws numbers and lays out primitive fields.  It holds none
of the scheme's arithmetic (no conversion to conserved variables, no fluxes,
no timestep); both the HIP path and the CPU oracle receive these primitive
fields and convert them with their own code.

Every generator returns a ``Workload`` with primitive fields
W = (rho, u, v, Pxx, Pxy, Pyy) as a float64 array [6, ny, nx] (1-D: [6, n])
plus the grid description.  Random numbers come from
``numpy.random.Generator(PCG64(seed))``.

"Smooth Gaussian field" (``smooth_gaussian``): iid N(0, 1) per cell,
periodic FFT convolution with a Gaussian kernel of standard deviation
``width`` cells, renormalised to zero mean and unit standard deviation.

The paper measures on no public dataset; these stand in for its workloads:

* ``sod``      -- the 1-D modified Sod tube of Sec. 4.1 (256 cells, t = 0.2);
* ``periodic`` -- a 2-D periodic random state (lognormal density, smooth
                  velocities, stress P = rho L L^T positive-definite);
* ``disc``     -- a 2-D galactic-disc-shaped state in the shape of Sec. 4.4
                  (exponential surface density, flat rotation curve held by a
                  fixed external potential, Toomre-Q dispersion, anisotropic
                  stress, m = 2 perturbation with phase noise);
* ``tubes``    -- many independent 1-D shock tubes of uneven length;
* ``adjoint``  -- the periodic generator at 512^2 plus the target's seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import ndtr

BC_PERIODIC = 0
BC_OUTFLOW = 1


@dataclass
class Workload:
    name: str
    W: np.ndarray            # primitive fields [6, ny, nx] or [6, n]
    nx: int
    ny: int
    dx: float
    dy: float
    bcx: int
    bcy: int
    x0: float = 0.0
    y0: float = 0.0
    vc: float = 0.0          # external flat-rotation-curve potential (0: none)
    rc: float = 0.0
    cfl: float = 0.8
    nsteps: int | None = None
    t_end: float | None = None
    extra: dict = field(default_factory=dict)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def smooth_gaussian(g: np.random.Generator, shape, width: float = 8.0) -> np.ndarray:
    """Periodic Gaussian-smoothed white noise, zero mean, unit std."""
    white = g.standard_normal(shape)
    ky = np.fft.fftfreq(shape[0])[:, None]
    kx = np.fft.rfftfreq(shape[1])[None, :]
    kernel_hat = np.exp(-2.0 * (math.pi * width) ** 2 * (kx * kx + ky * ky))
    f = np.fft.irfft2(np.fft.rfft2(white) * kernel_hat, s=shape)
    f -= f.mean()
    f /= f.std()
    return f


def sod(n: int = 256, t_end: float = 0.2) -> Workload:
    """1-D modified Sod tube: left (x < 0.5) rho = 1, Pxx = Pyy = 1; right
    rho = 0.125, Pxx = Pyy = 0.1; u = v = Pxy = 0; outflow on [0, 1]."""
    x = (np.arange(n) + 0.5) / n
    left = x < 0.5
    W = np.zeros((6, n))
    W[0] = np.where(left, 1.0, 0.125)
    W[3] = np.where(left, 1.0, 0.1)
    W[5] = np.where(left, 1.0, 0.1)
    return Workload("sod1d", W, n, 1, 1.0 / n, 1.0, BC_OUTFLOW, BC_OUTFLOW,
                    t_end=t_end, extra={"x": x})


def periodic(n: int = 1024, seed: int = 2, nsteps: int = 100) -> Workload:
    """2-D periodic random state on [0,1]^2.

    rho = exp(0.3 g1) (lognormal, mu 0, sigma 0.3, smoothed before
    exponentiation); u = 0.1 g2, v = 0.1 g3; L = [[L11, 0], [L21, L22]] with
    L11, L22 = 0.5 + 0.5 Phi(g4), 0.5 + 0.5 Phi(g5) and L21 = -0.2 + 0.4 Phi(g6)
    (exact uniform marginals); P = rho L L^T.  g_k are smooth Gaussian fields
    of width 8 cells drawn in that order.
    """
    g = rng(seed)
    shape = (n, n)
    gs = [smooth_gaussian(g, shape, 8.0) for _ in range(6)]
    rho = np.exp(0.3 * gs[0])
    l11 = 0.5 + 0.5 * ndtr(gs[3])
    l22 = 0.5 + 0.5 * ndtr(gs[4])
    l21 = -0.2 + 0.4 * ndtr(gs[5])
    W = np.stack([rho, 0.1 * gs[1], 0.1 * gs[2],
                  rho * l11 * l11, rho * l11 * l21, rho * (l21 * l21 + l22 * l22)])
    return Workload(f"periodic{n}", W, n, n, 1.0 / n, 1.0 / n, BC_PERIODIC, BC_PERIODIC,
                    nsteps=nsteps, extra={"seed": seed})


def disc(n: int = 4096, seed: int = 3, nsteps: int = 50, vc: float = 1.0, rc: float = 0.02,
         scale: float = 0.1, q_toomre: float = 1.5, sigma_floor: float = 0.02,
         anisotropy: float = 0.7, m2_amp: float = 0.01, phase_noise: float = 0.1) -> Workload:
    """2-D disc on the box [-1/2, 1/2]^2, outflow boundaries.

    Sigma = exp(-R / scale) (1 + m2_amp cos(2 phi + psi)), psi = phase_noise g;
    fixed potential of a flat rotation curve (circular speed vc, core rc),
    circular velocity vc R / sqrt(R^2 + rc^2); epicycle frequency of that
    potential kappa = vc sqrt(2 R^2 + 4 rc^2) / (R^2 + rc^2);
    sigma_R = max(3.36 Q G Sigma / kappa, sigma_floor) from the Toomre criterion
    (Sec. 4.4, eq. (39)) with Q = 1.5, G = 1; sigma_phi = 0.7 sigma_R;
    (P_RR, P_phiphi) = Sigma (sigma_R^2, sigma_phi^2) rotated to x, y.
    """
    g = rng(seed)
    dx = 1.0 / n
    c = -0.5 + (np.arange(n) + 0.5) * dx
    x = c[None, :]
    y = c[:, None]
    R2 = x * x + y * y
    R = np.sqrt(R2)
    phi = np.arctan2(y, x)
    psi = phase_noise * smooth_gaussian(g, (n, n), 8.0)
    sigma = np.exp(-R / scale) * (1.0 + m2_amp * np.cos(2.0 * phi + psi))
    vphi = vc * R / np.sqrt(R2 + rc * rc)
    kappa = vc * np.sqrt(2.0 * R2 + 4.0 * rc * rc) / (R2 + rc * rc)
    sig_r = np.maximum(3.36 * q_toomre * sigma / kappa, sigma_floor)
    sig_p = anisotropy * sig_r
    prr = sigma * sig_r ** 2
    ppp = sigma * sig_p ** 2
    cph, sph = np.cos(phi), np.sin(phi)
    W = np.stack([sigma, -vphi * sph, vphi * cph,
                  prr * cph * cph + ppp * sph * sph,
                  (prr - ppp) * sph * cph,
                  prr * sph * sph + ppp * cph * cph])
    return Workload(f"disc{n}", W, n, n, dx, dx, BC_OUTFLOW, BC_OUTFLOW, x0=-0.5, y0=-0.5,
                    vc=vc, rc=rc, nsteps=nsteps, extra={"seed": seed})


@dataclass
class Tubes:
    lengths: np.ndarray      # [ntubes] int64
    offsets: np.ndarray      # [ntubes + 1] int64, tube k = cells offsets[k]:offsets[k+1]
    W: np.ndarray            # primitive fields [6, sum(lengths)], tubes concatenated
    left: np.ndarray         # [ntubes, 4] (rho, u, Pxx, Pyy)
    right: np.ndarray
    cfl: float = 0.8
    nsteps: int = 200


def tubes(ntubes: int = 512, seed: int = 4, nmin: int = 128, nmax: int = 4096,
          nsteps: int = 200) -> Tubes:
    """Independent 1-D shock tubes on [0, 1] (dx = 1/N_k), discontinuity at 1/2,
    outflow ends.  Draw order: all lengths N_k ~ U{nmin..nmax}, then per tube
    the left state and the right state, each (rho ~ U(0.1, 1), u ~ U(-0.5, 0.5),
    Pxx ~ U(0.05, 1), Pyy ~ U(0.05, 1)); v = Pxy = 0.  Asserts that no tube
    would open a vacuum (gamma = 3: a_L + a_R > u_R - u_L)."""
    g = rng(seed)
    lengths = g.integers(nmin, nmax, size=ntubes, endpoint=True).astype(np.int64)
    left = np.empty((ntubes, 4))
    right = np.empty((ntubes, 4))
    for k in range(ntubes):
        for st in (left, right):
            st[k] = (g.uniform(0.1, 1.0), g.uniform(-0.5, 0.5),
                     g.uniform(0.05, 1.0), g.uniform(0.05, 1.0))
    aL = np.sqrt(3.0 * left[:, 2] / left[:, 0])
    aR = np.sqrt(3.0 * right[:, 2] / right[:, 0])
    assert np.all(aL + aR > right[:, 1] - left[:, 1]), "vacuum-generating tube drawn"
    offsets = np.zeros(ntubes + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    W = np.zeros((6, int(offsets[-1])))
    for k in range(ntubes):
        n = int(lengths[k])
        x = (np.arange(n) + 0.5) / n
        lft = x < 0.5
        sl = slice(int(offsets[k]), int(offsets[k + 1]))
        W[0, sl] = np.where(lft, left[k, 0], right[k, 0])
        W[1, sl] = np.where(lft, left[k, 1], right[k, 1])
        W[3, sl] = np.where(lft, left[k, 2], right[k, 2])
        W[5, sl] = np.where(lft, left[k, 3], right[k, 3])
    return Tubes(lengths, offsets, W, left, right, nsteps=nsteps)


def tube_workload(t: Tubes, k: int) -> Workload:
    n = int(t.lengths[k])
    W = np.ascontiguousarray(t.W[:, int(t.offsets[k]):int(t.offsets[k + 1])])
    return Workload(f"tube{k}", W, n, 1, 1.0 / n, 1.0, BC_OUTFLOW, BC_OUTFLOW,
                    cfl=t.cfl, nsteps=t.nsteps)


def adjoint(n: int = 512, seed: int = 5, target_seed: int = 6, nsteps: int = 200,
            checkpoint_every: int = 20):
    """(initial workload, target workload): the periodic generator at n^2 with
    ``seed``; the target density is the final density of a forward run from the
    generator with ``target_seed`` (the perturbed seed)."""
    w0 = periodic(n, seed, nsteps)
    wt = periodic(n, target_seed, nsteps)
    w0.name = f"adjoint{n}"
    w0.extra["checkpoint_every"] = checkpoint_every
    return w0, wt


def fd_directions(n: int, count: int = 64, base_seed: int = 1000) -> list:
    """Smooth random directions for the finite-difference check of the gradient:
    direction k draws six smooth fields (seed base_seed + k), each scaled to max-abs 1."""
    dirs = []
    for k in range(count):
        g = rng(base_seed + k)
        d = np.stack([smooth_gaussian(g, (n, n), 8.0) for _ in range(6)])
        d /= np.abs(d).max(axis=(1, 2), keepdims=True)
        dirs.append(d)
    return dirs


# ---- three dimensions ---------------------------------------------------------------------------

def smooth_gaussian3(g: np.random.Generator, shape, width: float = 4.0) -> np.ndarray:
    """3-D periodic Gaussian-smoothed white noise, zero mean, unit std."""
    white = g.standard_normal(shape)
    k0 = np.fft.fftfreq(shape[0])[:, None, None]
    k1 = np.fft.fftfreq(shape[1])[None, :, None]
    k2 = np.fft.rfftfreq(shape[2])[None, None, :]
    kernel_hat = np.exp(-2.0 * (math.pi * width) ** 2 * (k0 * k0 + k1 * k1 + k2 * k2))
    f = np.fft.irfftn(np.fft.rfftn(white) * kernel_hat, s=shape, axes=(0, 1, 2))
    f -= f.mean()
    f /= f.std()
    return f


@dataclass
class Workload3:
    name: str
    W: np.ndarray            # primitive fields [10, nz, ny, nx]:
                             # rho, u, v, w, Pxx, Pxy, Pxz, Pyy, Pyz, Pzz
    n: tuple                 # (nx, ny, nz)
    h: tuple                 # (dx, dy, dz)
    bc: tuple                # boundary kind per axis
    nsteps: int | None = None


def periodic3(nx: int = 64, ny: int | None = None, nz: int | None = None, seed: int = 7,
              nsteps: int = 20, width: float = 4.0) -> Workload3:
    """3-D periodic random state on [0,1]^3, the 2-D periodic recipe in three
    dimensions: rho = exp(0.3 g1), velocities 0.1 g2..g4, P = rho L L^T with
    L lower triangular, diagonal 0.5 + 0.5 Phi(g), off-diagonal -0.2 + 0.4 Phi(g)
    (g: smooth fields of width ``width`` cells)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    r = rng(seed)
    shape = (nz, ny, nx)
    gs = [smooth_gaussian3(r, shape, width) for _ in range(10)]
    W = np.empty((10,) + shape)
    W[0] = np.exp(0.3 * gs[0])
    W[1:4] = 0.1 * np.stack(gs[1:4])
    L = np.zeros((3, 3) + shape)
    L[0, 0] = 0.5 + 0.5 * ndtr(gs[4])
    L[1, 1] = 0.5 + 0.5 * ndtr(gs[5])
    L[2, 2] = 0.5 + 0.5 * ndtr(gs[6])
    L[1, 0] = -0.2 + 0.4 * ndtr(gs[7])
    L[2, 0] = -0.2 + 0.4 * ndtr(gs[8])
    L[2, 1] = -0.2 + 0.4 * ndtr(gs[9])
    P = np.einsum("ik...,jk...->ij...", L, L)
    for (i, j), m in zip(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)), range(4, 10)):
        W[m] = W[0] * P[i, j]
    return Workload3("periodic3d", W, (nx, ny, nz), (1.0 / nx, 1.0 / ny, 1.0 / nz),
                     (BC_PERIODIC,) * 3, nsteps)

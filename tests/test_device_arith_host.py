"""The sweep kernels' per-state arithmetic (csh_device.h, csh3_device.h, run
on the CPU by tests/host/device_host.hip) against the oracle's per-state
functions on random positive-definite states.

The kernels use closed forms the oracle does not: scaled characteristic
amplitudes with the MC limiter applied to them and the slope halved, the
limiter from order statistics, HLL and the KT flux formed from F - sU, the
tracing in the collapsed form.  The oracle uses dense eigenvector matrices and
the printed formulas.  Agreement to a few ulp of the data's scale on thousands
of states pins each closed form to its definition without a GPU."""
import ctypes
import os
import sys

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "host"))
import build_host  # noqa: E402

_D = ctypes.POINTER(ctypes.c_double)
_lib = None
N_STATES = 2000


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build_host.build_device())
        L.dev_mc_half.argtypes = [ctypes.c_double, ctypes.c_double]
        L.dev_mc_half.restype = ctypes.c_double
        for f in (L.dev_slope, L.dev_slope3):
            f.argtypes = [ctypes.c_int, _D, _D, _D, _D]
        for f in (L.dev_hll, L.dev_hllc, L.dev_kt_flux, L.dev_hll3):
            f.argtypes = [ctypes.c_int, _D, _D, _D]
        L.dev_faces_1d.argtypes = [_D, _D, _D, ctypes.c_double, _D, _D]
        _lib = L
    return _lib


def p(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(_D)


def states2(rng, n):
    """n random primitive states (rho, u, v, Pxx, Pxy, Pyy), P = rho L L^T."""
    rho = rng.uniform(0.1, 2.0, n)
    u, v = rng.uniform(-1.0, 1.0, (2, n))
    l11, l22 = rng.uniform(0.3, 1.2, (2, n))
    l21 = rng.uniform(-0.5, 0.5, n)
    return np.stack([rho, u, v, rho * l11 ** 2, rho * l11 * l21, rho * (l21 ** 2 + l22 ** 2)], axis=1)


def states3(rng, n):
    """n random 10-moment primitive states, P = rho L L^T with L lower triangular."""
    rho = rng.uniform(0.1, 2.0, n)
    vel = rng.uniform(-1.0, 1.0, (n, 3))
    L = np.zeros((n, 3, 3))
    L[:, [0, 1, 2], [0, 1, 2]] = rng.uniform(0.3, 1.2, (n, 3))
    L[:, [1, 2, 2], [0, 0, 1]] = rng.uniform(-0.5, 0.5, (n, 3))
    P = rho[:, None, None] * L @ L.transpose(0, 2, 1)
    idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    return np.concatenate([rho[:, None], vel, np.stack([P[:, i, j] for i, j in idx], axis=1)], axis=1)


def neighbours(rng, w, amp):
    """Two neighbouring states: w perturbed by relative noise of size amp (some
    components with opposite signs of their differences, so the limiter takes
    every branch)."""
    def pert():
        q = w * (1.0 + amp * rng.uniform(-1.0, 1.0, w.shape))
        q[:, 1:3] = w[:, 1:3] + amp * rng.uniform(-1.0, 1.0, w[:, 1:3].shape)
        return q
    return pert(), pert()


def close(got, ref, scale, rtol):
    return np.abs(got - ref).max() <= rtol * scale


def test_mc_half_is_half_the_limiter():
    rng = np.random.default_rng(41)
    vals = np.concatenate([rng.normal(size=3000), [0.0, -0.0, 1.0, -1.0, 2.0, 0.5]])
    f = lib().dev_mc_half
    for _ in range(4000):
        dl, dr = rng.choice(vals, 2)
        got = 2.0 * f(dl, dr)
        assert got == oracle.mc(dl, 0.5 * (dl + dr), dr), (dl, dr)


@pytest.mark.parametrize("direction", [0, 1])
def test_characteristic_slope(direction):
    rng = np.random.default_rng(42 + direction)
    w0 = states2(rng, N_STATES)
    wm, wp = neighbours(rng, w0, 0.3)
    got, worst = np.empty(6), 0.0
    for k in range(N_STATES):
        lib().dev_slope(direction, p(wm[k]), p(w0[k]), p(wp[k]), got.ctypes.data_as(_D))
        ref = oracle.limited_slope(direction, wm[k], w0[k], wp[k])
        scale = max(np.abs(wp[k] - w0[k]).max(), np.abs(w0[k] - wm[k]).max())
        worst = max(worst, np.abs(got - ref).max() / scale)
    assert worst <= 1e-12, worst


def test_face_states_1d():
    rng = np.random.default_rng(44)
    w0 = states2(rng, N_STATES)
    wl, wr = neighbours(rng, w0, 0.3)
    lo, hi = np.empty(6), np.empty(6)
    for k in range(N_STATES):
        kdt = rng.uniform(0.01, 0.2) / (np.abs(w0[k, 1]) + np.sqrt(3 * w0[k, 3] / w0[k, 0]))
        lib().dev_faces_1d(p(wl[k]), p(w0[k]), p(wr[k]), kdt, lo.ctypes.data_as(_D), hi.ctypes.data_as(_D))
        dwm = oracle.limited_slope(0, wl[k], w0[k], wr[k])
        rlo, rhi = oracle.trace(0, w0[k], dwm, kdt)
        scale = np.abs(w0[k]).max()
        assert close(lo, rlo, scale, 1e-13) and close(hi, rhi, scale, 1e-13), k


@pytest.mark.parametrize("solver", ["hll", "hllc", "kt"])
@pytest.mark.parametrize("direction", [0, 1])
def test_face_fluxes(solver, direction):
    rng = np.random.default_rng(45 + direction)
    wl = states2(rng, N_STATES)
    wr = np.where(rng.uniform(size=(N_STATES, 1)) < 0.5, neighbours(rng, wl, 0.2)[0], states2(rng, N_STATES))
    dev = {"hll": lib().dev_hll, "hllc": lib().dev_hllc, "kt": lib().dev_kt_flux}[solver]
    ref_f = {"hll": oracle.hll, "hllc": oracle.hllc, "kt": oracle.kt_flux}[solver]
    got = np.empty(6)
    for k in range(N_STATES):
        dev(direction, p(wl[k]), p(wr[k]), got.ctypes.data_as(_D))
        ref = ref_f(direction, wl[k], wr[k])
        scale = max(np.abs(oracle.flux(direction, oracle.cons(w))).max() for w in (wl[k], wr[k]))
        assert close(got, ref, scale, 1e-13), (solver, k, got, ref)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_characteristic_slope_3d(axis):
    rng = np.random.default_rng(48 + axis)
    n = N_STATES // 2
    w0 = states3(rng, n)
    wm, wp = neighbours(rng, w0, 0.3)
    got, worst = np.empty(10), 0.0
    for k in range(n):
        lib().dev_slope3(axis, p(wm[k]), p(w0[k]), p(wp[k]), got.ctypes.data_as(_D))
        ref = oracle.limited_slope3(axis, wm[k], w0[k], wp[k])
        scale = max(np.abs(wp[k] - w0[k]).max(), np.abs(w0[k] - wm[k]).max())
        worst = max(worst, np.abs(got - ref).max() / scale)
    assert worst <= 1e-12, worst


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hll_3d(axis):
    rng = np.random.default_rng(51 + axis)
    n = N_STATES // 2
    wl, wr = states3(rng, n), states3(rng, n)
    got = np.empty(10)
    for k in range(n):
        lib().dev_hll3(axis, p(wl[k]), p(wr[k]), got.ctypes.data_as(_D))
        ref = oracle.hll3(axis, wl[k], wr[k])
        scale = max(np.abs(oracle.flux3(axis, oracle.cons3(w))).max() for w in (wl[k], wr[k]))
        assert close(got, ref, scale, 1e-13), (k, got, ref)


# ---- the device's reciprocal and square roots ------------------------------------------------

def _exact(fn, x):
    """fn(x) rounded from an exact rational (or a double-double square root)."""
    from fractions import Fraction
    import decimal
    if fn == "rcp":
        return Fraction(1) / Fraction(x)
    ctx = decimal.Context(prec=60)
    r = decimal.Decimal(x).sqrt(ctx)
    return Fraction(r) if fn == "sqrt" else Fraction(1) / Fraction(r)


@pytest.mark.parametrize("fn,bound", [("rcp", 4e-15), ("rsqrt", 6e-15), ("sqrt", 6e-15)])
def test_newton_refinement_from_hardware_accuracy(fn, bound):
    """On the GPU the reciprocal and square roots are the hardware's FP64
    approximation (measured ~5e-8 relative on gfx950) refined by one Newton
    step.  The refinement code itself, run here from approximations 6e-8 off
    in either direction (and at random within that), lands within the bound on
    x across 1e-200..1e200: the error squares (x 3/2 for the roots), plus the
    step's own rounding."""
    from fractions import Fraction
    f = {"rcp": lib().dev_rcp_refine, "rsqrt": lib().dev_rsqrt_refine, "sqrt": lib().dev_sqrt_refine}[fn]
    f.argtypes = [ctypes.c_double, ctypes.c_double]
    f.restype = ctypes.c_double
    r = np.random.default_rng(77)
    xs = np.concatenate([10.0 ** r.uniform(-200, 200, 300), r.uniform(0.5, 2.0, 300), [1.0, 3.0, 0.1, 1e-300 * 1e100]])
    worst = 0.0
    for x in xs:
        x = float(x)
        # the approximation the refinement starts from: of 1/x for rcp, of 1/sqrt(x) for both roots
        target = _exact("rcp", x) if fn == "rcp" else _exact("rsqrt", x)
        for e in (6e-8, -6e-8, float(r.uniform(-6e-8, 6e-8))):
            approx = float(target * (1 + Fraction(e)))
            got = Fraction(f(x, approx))
            want = _exact(fn, x)
            worst = max(worst, float(abs(got - want) / want))
    assert worst <= bound, worst

"""FP64 CPU oracle for the collisionless-stellar-hydrodynamics sweep.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP implementation in ``paper_1210_5246_amd``; neither imports the
other.

The arithmetic lives in ``cshoracle.c`` (plain C, FP64, built by the host
compiler with ``-O2 -ffp-contract=off``, no fast-math, OpenMP over rows).
This module is the ctypes shim plus a few time loops written directly from the
paper:

* ``run_cfl``        -- the time loop: dt = C / s from the state at the start
                        of each step (the paper gives no formula; reading R8 of
                        ``cshoracle.c``), optionally clipped to an end time;
* ``dense_jacobian`` -- brute-force central-difference Jacobian of one step at
                        frozen dt (used to pin the adjoint).

Arrays are numpy float64, structure-of-arrays ``[6, ny, nx]`` (1-D: ``[6, n]``),
conserved U = (rho, rho u, rho v, Exx, Exy, Eyy), primitive
W = (rho, u, v, Pxx, Pxy, Pyy).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cshoracle.c")
_SRC3 = os.path.join(_HERE, "cshoracle3.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# A test may point the shim at a differently built copy (planted-mistake checks).
_LIB_OVERRIDE = os.environ.get("CSH_ORACLE_LIB")

BC_PERIODIC = 0
BC_OUTFLOW = 1


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (gcc)."""
    newest = max(os.path.getmtime(f) for f in (_SRC, _SRC3))
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c99", "-Wall", "-o", tmp, _SRC, _SRC3, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("bcx", ctypes.c_int), ("bcy", ctypes.c_int),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("vc", ctypes.c_double), ("rc", ctypes.c_double)]


@dataclass
class Grid:
    """Uniform grid.  ny == 1 selects the 1-D scheme."""
    nx: int
    ny: int = 1
    dx: float = 1.0
    dy: float = 1.0
    bcx: int = BC_PERIODIC
    bcy: int = BC_PERIODIC
    x0: float = 0.0
    y0: float = 0.0
    vc: float = 0.0   # flat-rotation-curve external potential (0: none)
    rc: float = 0.0

    def c(self) -> _Grid:
        return _Grid(self.nx, self.ny, self.dx, self.dy, self.bcx, self.bcy,
                     self.x0, self.y0, self.vc, self.rc)


class _Grid3(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("h", ctypes.c_double * 3), ("bc", ctypes.c_int * 3)]


@dataclass
class Grid3:
    """Uniform 3-D grid: cells (nx, ny, nz), sizes (dx, dy, dz), boundary kinds per axis."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    bc: tuple = (BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)

    def c(self) -> _Grid3:
        return _Grid3((ctypes.c_int * 3)(self.nx, self.ny, self.nz),
                      (ctypes.c_double * 3)(self.dx, self.dy, self.dz),
                      (ctypes.c_int * 3)(*self.bc))


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
                    os.path.getmtime(_SRC), os.path.getmtime(_SRC3)):
                build(force=True)
            L = ctypes.CDLL(_LIB_PATH)
        G = ctypes.POINTER(_Grid)
        L.orc_step.argtypes = [G, ctypes.c_double, _D, _D]
        L.orc_step_cells.argtypes = [G, ctypes.c_double, _D, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64), _D]
        L.orc_fluxes.argtypes = [G, ctypes.c_double, _D, _D, _D]
        L.orc_max_signal_speed.argtypes = [G, _D]
        L.orc_max_signal_speed.restype = ctypes.c_double
        L.orc_physical.argtypes = [G, _D]
        L.orc_branch_count.argtypes = [G]
        L.orc_branch_count.restype = ctypes.c_int64
        L.orc_branches.argtypes = [G, ctypes.c_double, _D, ctypes.POINTER(ctypes.c_int)]
        L.orc_cons_field.argtypes = [ctypes.c_int64, _D, _D]
        L.orc_prim_field.argtypes = [ctypes.c_int64, _D, _D]
        for name in ("orc_cons", "orc_prim", "orc_flux_x", "orc_flux_y"):
            getattr(L, name).argtypes = [_D, _D]
        for name in ("orc_jac_x", "orc_jac_y"):
            getattr(L, name).argtypes = [_D, _D]
        for name in ("orc_eigen_x", "orc_eigen_y"):
            getattr(L, name).argtypes = [_D, _D, _D, _D]
        L.orc_mc.argtypes = [ctypes.c_double] * 3
        L.orc_mc.restype = ctypes.c_double
        L.orc_limited_slope.argtypes = [ctypes.c_int, _D, _D, _D, _D]
        L.orc_trace.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double, _D, _D]
        L.orc_hll.argtypes = [ctypes.c_int, _D, _D, _D]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_kt_flux.argtypes = [ctypes.c_int, _D, _D, _D]
        L.orc_step_kt.argtypes = [G, ctypes.c_double, _D, _D]
        L.orc_hllc.argtypes = [ctypes.c_int, _D, _D, _D]
        L.orc_hllc_star.argtypes = [ctypes.c_int, _D, _D, _D, _D, _D]
        L.orc_step_rs.argtypes = [G, ctypes.c_int, ctypes.c_double, _D, _D]
        L.orc_step_cells_rs.argtypes = [G, ctypes.c_int, ctypes.c_double, _D, ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_int64), _D]
        L.orc_fluxes_rs.argtypes = [G, ctypes.c_int, ctypes.c_double, _D, _D, _D]
        G3 = ctypes.POINTER(_Grid3)
        for name in ("orc3_cons", "orc3_prim"):
            getattr(L, name).argtypes = [_D, _D]
        L.orc3_flux.argtypes = [ctypes.c_int, _D, _D]
        L.orc3_jac.argtypes = [ctypes.c_int, _D, _D]
        L.orc3_eigen.argtypes = [ctypes.c_int, _D, _D, _D, _D]
        L.orc3_limited_slope.argtypes = [ctypes.c_int, _D, _D, _D, _D]
        L.orc3_trace.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double, _D, _D]
        L.orc3_hll.argtypes = [ctypes.c_int, _D, _D, _D]
        L.orc3_step.argtypes = [G3, ctypes.c_double, _D, _D]
        L.orc3_step_cells.argtypes = [G3, ctypes.c_double, _D, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _D]
        L.orc3_max_signal_speed.argtypes = [G3, _D]
        L.orc3_max_signal_speed.restype = ctypes.c_double
        L.orc_fourier_amplitudes.argtypes = [G, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _vec(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


# ---- pointwise pieces (for the pin tests) -------------------------------------------

def cons(w) -> np.ndarray:
    w = _vec(w); out = np.empty(6); lib().orc_cons(_p(w), _p(out)); return out


def prim(U) -> np.ndarray:
    U = _vec(U); out = np.empty(6); lib().orc_prim(_p(U), _p(out)); return out


def flux(direction: int, U) -> np.ndarray:
    U = _vec(U); out = np.empty(6)
    (lib().orc_flux_x if direction == 0 else lib().orc_flux_y)(_p(U), _p(out))
    return out


def jacobian(direction: int, w) -> np.ndarray:
    w = _vec(w); out = np.empty((6, 6))
    (lib().orc_jac_x if direction == 0 else lib().orc_jac_y)(_p(w), _p(out))
    return out


def eigen(direction: int, w):
    """(lam[6], R[6,6] with eigenvectors in columns, L[6,6] with them in rows)."""
    w = _vec(w); lam = np.empty(6); R = np.empty((6, 6)); L = np.empty((6, 6))
    (lib().orc_eigen_x if direction == 0 else lib().orc_eigen_y)(_p(w), _p(lam), _p(R), _p(L))
    return lam, R, L


def mc(dl: float, dc: float, dr: float) -> float:
    return lib().orc_mc(dl, dc, dr)


def limited_slope(direction: int, wm, w0, wp) -> np.ndarray:
    wm, w0, wp = _vec(wm), _vec(w0), _vec(wp); out = np.empty(6)
    lib().orc_limited_slope(direction, _p(wm), _p(w0), _p(wp), _p(out))
    return out


def trace(direction: int, w, dwm, k: float):
    """(w_lo, w_hi): states on the low (i-1/2) and high (i+1/2) faces."""
    w, dwm = _vec(w), _vec(dwm); lo = np.empty(6); hi = np.empty(6)
    lib().orc_trace(direction, _p(w), _p(dwm), k, _p(lo), _p(hi))
    return lo, hi


def hll(direction: int, wl, wr) -> np.ndarray:
    wl, wr = _vec(wl), _vec(wr); out = np.empty(6)
    lib().orc_hll(direction, _p(wl), _p(wr), _p(out))
    return out


def hllc(direction: int, wl, wr) -> np.ndarray:
    """HLLC flux of the BME (reading H1 in cshoracle.c)."""
    wl, wr = _vec(wl), _vec(wr); out = np.empty(6)
    lib().orc_hllc(direction, _p(wl), _p(wr), _p(out))
    return out


def hllc_star(direction: int, wl, wr):
    """(S_L, S*, S_R), U*_L, U*_R of the HLLC fan."""
    wl, wr = _vec(wl), _vec(wr)
    S, UsL, UsR = np.empty(3), np.empty(6), np.empty(6)
    lib().orc_hllc_star(direction, _p(wl), _p(wr), _p(S), _p(UsL), _p(UsR))
    return S, UsL, UsR


SOLVERS = {"hll": 0, "hllc": 1}


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Set the OpenMP threads of the oracle's loops (the CPU baseline's 1-thread leg)."""
    lib().orc_set_num_threads(int(n))


# ---- fields ----------------------------------------------------------------------------

def cons_field(W: np.ndarray) -> np.ndarray:
    W = np.ascontiguousarray(W, dtype=np.float64)
    U = np.empty_like(W)
    lib().orc_cons_field(W[0].size, _p(W), _p(U))
    return U


def prim_field(U: np.ndarray) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    W = np.empty_like(U)
    lib().orc_prim_field(U[0].size, _p(U), _p(W))
    return W


def _check(g: Grid, U: np.ndarray) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    if U.size != 6 * g.nx * g.ny:
        raise ValueError("state has the wrong size for the grid")
    return U


def step(g: Grid, dt: float, U: np.ndarray, solver: str = "hll") -> np.ndarray:
    """One step of the characteristic scheme (Sec. 3.3) with an HLL or HLLC flux."""
    U = _check(g, U); out = np.empty_like(U)
    if lib().orc_step_rs(ctypes.byref(g.c()), SOLVERS[solver], dt, _p(U), _p(out)) != 0:
        raise ValueError("bad grid")
    return out


def kt_flux(direction: int, wl, wr) -> np.ndarray:
    """Numerical flux of eq. (6) of the Kurganov-Tadmor scheme (u^- = wl, u^+ = wr)."""
    wl, wr = _vec(wl), _vec(wr); out = np.empty(6)
    lib().orc_kt_flux(direction, _p(wl), _p(wr), _p(out))
    return out


def step_kt(g: Grid, dt: float, U: np.ndarray) -> np.ndarray:
    """One step of the Kurganov-Tadmor scheme (Sec. 3.2; readings in cshoracle.c)."""
    U = _check(g, U); out = np.empty_like(U)
    if lib().orc_step_kt(ctypes.byref(g.c()), dt, _p(U), _p(out)) != 0:
        raise ValueError("bad grid")
    return out


# ---- three dimensions (cshoracle3.c) ---------------------------------------------------

def cons3(w) -> np.ndarray:
    w = _vec(w); out = np.empty(10); lib().orc3_cons(_p(w), _p(out)); return out


def prim3(U) -> np.ndarray:
    U = _vec(U); out = np.empty(10); lib().orc3_prim(_p(U), _p(out)); return out


def flux3(axis: int, U) -> np.ndarray:
    U = _vec(U); out = np.empty(10); lib().orc3_flux(axis, _p(U), _p(out)); return out


def jac3(axis: int, w) -> np.ndarray:
    w = _vec(w); A = np.empty((10, 10)); lib().orc3_jac(axis, _p(w), _p(A)); return A


def eigen3(axis: int, w):
    """(lambda [10], R [10,10] right eigenvectors as columns, L = R^-1)."""
    w = _vec(w); lam, R, L = np.empty(10), np.empty((10, 10)), np.empty((10, 10))
    if lib().orc3_eigen(axis, _p(w), _p(lam), _p(R), _p(L)) != 1:
        raise ValueError("singular eigenvector matrix")
    return lam, R, L


def limited_slope3(axis: int, wm, w0, wp) -> np.ndarray:
    out = np.empty(10)
    lib().orc3_limited_slope(axis, _p(_vec(wm)), _p(_vec(w0)), _p(_vec(wp)), _p(out))
    return out


def trace3(axis: int, w, dw, k: float):
    lo, hi = np.empty(10), np.empty(10)
    lib().orc3_trace(axis, _p(_vec(w)), _p(_vec(dw)), float(k), _p(lo), _p(hi))
    return lo, hi


def hll3(axis: int, wl, wr) -> np.ndarray:
    out = np.empty(10); lib().orc3_hll(axis, _p(_vec(wl)), _p(_vec(wr)), _p(out)); return out


def _check3(g: Grid3, U: np.ndarray) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    if U.size != 10 * g.nx * g.ny * g.nz:
        raise ValueError("state has the wrong size for the grid")
    return U


_PIDX3 = ((4, 5, 6), (5, 7, 8), (6, 8, 9))


def cons3_field(W: np.ndarray) -> np.ndarray:
    """Primitive [10, ...] -> conserved [10, ...]: E_ij = P_ij + rho u_i u_j (Sec. 2)."""
    W = np.asarray(W, dtype=np.float64)
    U = np.empty_like(W)
    U[0] = W[0]
    for i in range(3):
        U[1 + i] = W[0] * W[1 + i]
        for j in range(i, 3):
            U[_PIDX3[i][j]] = W[_PIDX3[i][j]] + W[0] * W[1 + i] * W[1 + j]
    return U


def prim3_field(U: np.ndarray) -> np.ndarray:
    U = np.asarray(U, dtype=np.float64)
    W = np.empty_like(U)
    W[0] = U[0]
    for i in range(3):
        W[1 + i] = U[1 + i] / U[0]
    for i in range(3):
        for j in range(i, 3):
            W[_PIDX3[i][j]] = U[_PIDX3[i][j]] - U[0] * W[1 + i] * W[1 + j]
    return W


def step3(g: Grid3, dt: float, U: np.ndarray) -> np.ndarray:
    """One step of the 3-D characteristic scheme with HLL fluxes; U [10, nz, ny, nx]."""
    U = _check3(g, U); out = np.empty_like(U)
    if lib().orc3_step(ctypes.byref(g.c()), dt, _p(U), _p(out)) != 0:
        raise ValueError("bad grid")
    return out


def step3_cells(g: Grid3, dt: float, U: np.ndarray, cells) -> np.ndarray:
    """Updated states of the listed cells (flat index (k ny + j) nx + i): [len(cells), 10]."""
    U = _check3(g, U)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.empty((cells.size, 10))
    if lib().orc3_step_cells(ctypes.byref(g.c()), dt, _p(U), cells.size,
                             cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(out)) != 0:
        raise ValueError("bad grid")
    return out


def max_signal_speed3(g: Grid3, U: np.ndarray) -> float:
    return lib().orc3_max_signal_speed(ctypes.byref(g.c()), _p(_check3(g, U)))


def run_cfl3(g: Grid3, U: np.ndarray, nsteps: int, cfl: float = 0.8):
    """nsteps 3-D steps with dt = cfl / s from the state at the start of each step."""
    U = _check3(g, U).copy()
    dts = []
    for _ in range(nsteps):
        dt = cfl / max_signal_speed3(g, U)
        if not (dt > 0.0 and dt < float("inf")):
            raise FloatingPointError(f"timestep {dt}: the state is not physical")
        U = step3(g, dt, U)
        dts.append(dt)
    return U, dts


def fourier_amplitudes(g: Grid, U: np.ndarray, m_max: int = 6, X: float = float("inf"),
                       Y: float = float("inf")) -> np.ndarray:
    """Global Fourier amplitudes A_1..A_m_max of the density of a 2-D state
    (Sec. 4.4; readings F1-F3 in cshoracle.c) over the region [-X, X] x [-Y, Y]."""
    U = _check(g, U); out = np.empty(m_max)
    if lib().orc_fourier_amplitudes(ctypes.byref(g.c()), _p(U), int(m_max), float(X), float(Y), _p(out)) != 0:
        raise ValueError("bad grid (2-D only) or m_max < 1")
    return out


def step_cells(g: Grid, dt: float, U: np.ndarray, cells, solver: str = "hll") -> np.ndarray:
    """Updated conserved state of the listed cells (flat index j*nx+i): [len(cells), 6]."""
    U = _check(g, U)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.empty((cells.size, 6))
    if lib().orc_step_cells_rs(ctypes.byref(g.c()), SOLVERS[solver], dt, _p(U), cells.size,
                               cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(out)) != 0:
        raise ValueError("bad grid")
    return out


def fluxes(g: Grid, dt: float, U: np.ndarray, solver: str = "hll"):
    """(Fx [6, ny, nx+1], Fy [6, ny+1, nx] or None in 1-D)."""
    U = _check(g, U)
    Fx = np.empty((6, g.ny, g.nx + 1))
    Fy = np.empty((6, g.ny + 1, g.nx)) if g.ny > 1 else np.empty(6)
    if lib().orc_fluxes_rs(ctypes.byref(g.c()), SOLVERS[solver], dt, _p(U), _p(Fx), _p(Fy)) != 0:
        raise ValueError("bad grid")
    return Fx, (Fy if g.ny > 1 else None)


def max_signal_speed(g: Grid, U: np.ndarray) -> float:
    U = _check(g, U)
    return lib().orc_max_signal_speed(ctypes.byref(g.c()), _p(U))


def physical(g: Grid, U: np.ndarray) -> bool:
    U = _check(g, U)
    return bool(lib().orc_physical(ctypes.byref(g.c()), _p(U)))


MC_OFF, MC_CENTRED, MC_LEFT, MC_RIGHT = 0, 1, 2, 3


def branches(g: Grid, dt: float, U: np.ndarray) -> dict:
    """Branch pattern of one step (``orc_branches``): the side of every kink
    of the scheme that each decision takes.

    ``cells``: [ey, ex, 16] over the extended cells (j = -1..ny in 2-D, i =
    -1..nx): per direction x then y, the limiter code of each of the six waves
    (MC_OFF at an extremum, else MC_CENTRED / MC_LEFT / MC_RIGHT for the first
    minimal argument of |dc|, 2|dl|, 2|dr|) and the tracing kinks
    (lamM > 0, lam0 < 0); ``fx``: [ny, nx+1, 4] per x face i-1/2 and ``fy``
    [ny+1, nx, 4] per y face (2-D): which face state sets S_L, S_L >= 0, which
    sets S_R, S_R <= 0.
    """
    U = _check(g, U)
    n = int(lib().orc_branch_count(ctypes.byref(g.c())))
    codes = np.zeros(n, dtype=np.intc)
    if lib().orc_branches(ctypes.byref(g.c()), dt, _p(U), codes.ctypes.data_as(ctypes.POINTER(ctypes.c_int))) != 0:
        raise ValueError("bad grid")
    twod = g.ny > 1
    ex, ey = g.nx + 2, (g.ny + 2 if twod else 1)
    nc = 16 * ex * ey
    nfx = 4 * (g.nx + 1) * g.ny
    out = {"cells": codes[:nc].reshape(ey, ex, 16), "fx": codes[nc:nc + nfx].reshape(g.ny, g.nx + 1, 4)}
    if twod:
        out["fy"] = codes[nc + nfx:].reshape(g.ny + 1, g.nx, 4)
    return out


def same_branches(a: dict, b: dict) -> bool:
    return all(np.array_equal(a[k], b[k]) for k in a)


# ---- time loops ------------------------------------------------------------------------

def run_cfl(g: Grid, U: np.ndarray, nsteps: int | None = None, cfl: float = 0.8,
            t_end: float | None = None, max_steps: int = 20000, scheme: str = "muscl"):
    """Advance with dt = cfl / s (s from the state at the start of each step).

    Stops after ``nsteps`` steps, or when ``t_end`` is reached (the last step is
    clipped to land on it).  ``scheme``: "muscl" (Sec. 3.3, HLL flux), "hllc"
    (Sec. 3.3 with the HLLC flux) or "kt" (Sec. 3.2).
    Returns (U, list of dt).
    """
    U = _check(g, U).copy()
    dts, t = [], 0.0
    while True:
        if nsteps is not None and len(dts) >= nsteps:
            break
        if t_end is not None and t >= t_end:
            break
        if len(dts) >= max_steps:
            raise RuntimeError("too many steps")
        dt = cfl / max_signal_speed(g, U)
        if not (dt > 0.0 and dt < float("inf")):
            raise FloatingPointError(f"timestep {dt} at step {len(dts)}: the state is not physical")
        if t_end is not None and t + dt > t_end:
            dt = t_end - t
        if scheme == "kt":
            U = step_kt(g, dt, U)
        else:
            U = step(g, dt, U, "hllc" if scheme == "hllc" else "hll")
        dts.append(dt)
        t += dt
    return U, dts


def run_dts(g: Grid, U: np.ndarray, dts) -> np.ndarray:
    """Advance with a given list of timesteps."""
    U = _check(g, U).copy()
    for dt in dts:
        U = step(g, dt, U)
    return U


def dense_jacobian(g: Grid, dt: float, U: np.ndarray, rel: float = 1e-7, floor: float = 1e-3):
    """J[a, b] = d step(U)_a / d U_b by central differences at frozen dt.

    The step of component b is h_b = rel * max(|U_b|, floor).
    Flattened SoA order (the order of ``U.ravel()``).
    """
    U = _check(g, U)
    flat = U.ravel()
    n = flat.size
    J = np.empty((n, n))
    for b in range(n):
        h = rel * max(abs(flat[b]), floor)
        up = flat.copy(); up[b] += h
        dn = flat.copy(); dn[b] -= h
        J[:, b] = (step(g, dt, up.reshape(U.shape)).ravel()
                   - step(g, dt, dn.reshape(U.shape)).ravel()) / (2.0 * h)
    return J

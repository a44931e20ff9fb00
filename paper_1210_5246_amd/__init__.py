"""cshydro on MI355X: collisionless stellar hydrodynamics (arXiv:1210.5246).

Thin Python binding of the C ABI in ``include/cshydro.h`` (same names).  It
only marshals arguments: every step of the sweep runs in the HIP kernels of
``libcshydro.so``, built in-tree by ``paper_1210_5246_amd.build``.  PyTorch
provides device memory (tensors) and the stream (the current stream when a
handle is created).  There is no CPU fallback: without the built library or a
GPU, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcshydro.so")

CSH_OK = 0
CSH_ERR_ARG = -1
CSH_ERR_HIP = -2
CSH_ERR_NONPHYSICAL = -3
BC_PERIODIC = 0
BC_OUTFLOW = 1
F64 = 0
F32 = 1
SCHEMES = {"muscl": 0, "kt": 1, "hllc": 2}


class CshError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cshydro error {code}: {msg}")
        self.code = code


class NonPhysicalState(CshError):
    pass


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)

# (name, restype, argtypes) of every exported entry point
_SIGNATURES = [
    ("csh_last_error", ctypes.c_char_p, []),
    ("csh3_last_error", ctypes.c_char_p, []),
    ("csh3_init_state", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    ("csh3_step", ctypes.c_int, [_vp, ctypes.c_double, _vp, _vp]),
    ("csh3_max_signal_speed", ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_double)]),
    ("csh3_last_signal_speed", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double)]),
    ("csh3_run_cfl", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, _vp, _vp, _vp]),
    ("csh3_destroy", None, [_vp]),
    ("csh_init_state", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    ("csh_set_state", ctypes.c_int, [_vp, _vp, _vp]),
    ("csh_set_scheme", ctypes.c_int, [_vp, ctypes.c_int]),
    ("csh_fourier_amplitudes", ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    ("csh_fourier_amplitudes_noalloc", ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.c_double,
                                                      ctypes.c_double, ctypes.c_double, ctypes.c_int, _vp]),
    ("csh_set_potential", ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    ("csh_step", ctypes.c_int, [_vp, ctypes.c_double, _vp, _vp]),
    ("csh_max_signal_speed", ctypes.c_int, [_vp, _vp, _dp]),
    ("csh_last_signal_speed", ctypes.c_int, [_vp, _dp]),
    ("csh_fluxes", ctypes.c_int, [_vp, ctypes.c_double, _vp, _vp, _vp]),
    ("csh_run_cfl", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, _vp, _vp, _vp]),
    ("csh_run_cfl_states", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, _vp, _vp, _vp]),
    ("csh_run_dts", ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
    ("csh_adjoint_step", ctypes.c_int, [_vp, ctypes.c_double, _vp, _vp, _vp]),
    ("csh_init_state_adjoint", ctypes.c_int, [_vp, _vp, _vp, _vp]),
    ("csh_destroy", ctypes.c_int, [_vp]),
    ("csh_batch_init", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int, _vp, _vp, _vp]),
    ("csh_batch_run", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, _vp, _vp, _vp, ctypes.c_int]),
    ("csh_batch_autotune", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, _vp, ctypes.POINTER(ctypes.c_int)]),
    ("csh_batch_status", ctypes.c_int, [_vp]),
    ("csh_batch_destroy", ctypes.c_int, [_vp]),
]


def lib():
    """The loaded HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1210_5246_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code != CSH_OK:
        msg = lib().csh_last_error().decode(errors="replace")
        if code == CSH_ERR_NONPHYSICAL:
            raise NonPhysicalState(code, msg)
        raise CshError(code, msg)


def _dev(t: torch.Tensor, dtype, numel: int | None = None, at_least: bool = False) -> int:
    """Device pointer of a contiguous GPU tensor of ``dtype``; with ``numel``
    the tensor must hold exactly (``at_least``: at least) that many elements,
    since the kernels index it from the handle's sizes alone."""
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype} GPU tensor, got {t.dtype} on {t.device}")
    if numel is not None and (t.numel() < numel if at_least else t.numel() != numel):
        raise ValueError(f"expected {'at least ' if at_least else ''}{numel} elements, got {t.numel()}")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Grid:
    """A grid handle (``csh_grid``) plus the conserved state tensor ``U``.

    ``W``: primitive fields (rho, u, v, Pxx, Pxy, Pyy) as a contiguous GPU
    tensor [6, ny, nx] (2-D) or [6, n] (1-D), float64 or float32.
    """

    def __init__(self, W: torch.Tensor, dx: float, dy: float = 1.0,
                 bc=(BC_PERIODIC, BC_PERIODIC), check: bool = True):
        if W.dim() == 2:
            ny, nx = 1, W.shape[1]
        elif W.dim() == 3:
            ny, nx = W.shape[1], W.shape[2]
        else:
            raise ValueError("W must be [6, n] or [6, ny, nx]")
        if W.shape[0] != 6:
            raise ValueError("W must have 6 fields")
        self.dtype = W.dtype
        self.code = F64 if W.dtype == torch.float64 else F32
        self.shape = tuple(W.shape)
        self.nx, self.ny, self.dx, self.dy = nx, ny, float(dx), float(dy)
        self.U = torch.empty_like(W)
        self.n = 6 * nx * ny  # elements of a state
        self._h = _vp()
        code = lib().csh_init_state(ctypes.byref(self._h), nx, ny, self.dx, self.dy, int(bc[0]), int(bc[1]),
                                    self.code, _dev(W, W.dtype), _dev(self.U, W.dtype), _stream())
        if code == CSH_ERR_NONPHYSICAL and not check:
            return
        _check(code)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.csh_destroy(h)
            self._h = None

    # -- the C entry points -----------------------------------------------------------
    def set_state(self, W: torch.Tensor, U: torch.Tensor | None = None) -> torch.Tensor:
        """Primitive fields -> conserved state (default into ``self.U``) on this handle."""
        U = self.U if U is None else U
        _check(lib().csh_set_state(self._h, _dev(W, self.dtype, self.n), _dev(U, self.dtype, self.n)))
        return U

    def set_scheme(self, scheme: str):
        """"muscl" (characteristic MUSCL-Hancock + HLL, default), "hllc" (the same sweep with
        the HLLC flux) or "kt" (Kurganov-Tadmor)."""
        _check(lib().csh_set_scheme(self._h, SCHEMES[scheme]))

    def fourier_amplitudes(self, x0: float, y0: float, m_max: int = 6, X: float = float("inf"),
                           Y: float = float("inf"), U: torch.Tensor | None = None) -> list[float]:
        """Global Fourier amplitudes A_1..A_m_max of the density (``csh_fourier_amplitudes``);
        (x0, y0) is the lower-left corner of the grid, the region [-X, X] x [-Y, Y]."""
        U = self.U if U is None else U
        out = (ctypes.c_double * m_max)()
        _check(lib().csh_fourier_amplitudes(self._h, _dev(U, self.dtype, self.n), float(x0), float(y0), float(X), float(Y),
                                            int(m_max), out))
        return list(out)

    def fourier_amplitudes_noalloc(self, x0: float, y0: float, A: torch.Tensor, X: float = float("inf"),
                                   Y: float = float("inf"), U: torch.Tensor | None = None) -> torch.Tensor:
        """``csh_fourier_amplitudes_noalloc``: A_1..A_m (m = A.numel()) into the
        caller's float64 GPU tensor ``A``, in stream order, with no allocation."""
        U = self.U if U is None else U
        _check(lib().csh_fourier_amplitudes_noalloc(self._h, _dev(U, self.dtype, self.n), float(x0), float(y0),
                                                    float(X), float(Y), int(A.numel()), _dev(A, torch.float64)))
        return A

    def set_potential(self, vc: float, rc: float, x0: float, y0: float = 0.0):
        _check(lib().csh_set_potential(self._h, vc, rc, x0, y0))

    def step(self, dt: float, U: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
        """One sweep; returns the new state (a new tensor unless ``out`` is given)."""
        U = self.U if U is None else U
        out = torch.empty_like(U) if out is None else out
        _check(lib().csh_step(self._h, float(dt), _dev(U, self.dtype, self.n), _dev(out, self.dtype, self.n)))
        return out

    def max_signal_speed(self, U: torch.Tensor | None = None) -> float:
        U = self.U if U is None else U
        s = ctypes.c_double()
        _check(lib().csh_max_signal_speed(self._h, _dev(U, self.dtype, self.n), ctypes.byref(s)))
        return s.value

    def last_signal_speed(self) -> float:
        s = ctypes.c_double()
        _check(lib().csh_last_signal_speed(self._h, ctypes.byref(s)))
        return s.value

    def fluxes(self, dt: float, U: torch.Tensor | None = None):
        """(Fx [6, ny, nx+1], Fy [6, ny+1, nx] or None in 1-D)."""
        U = self.U if U is None else U
        Fx = torch.empty((6, self.ny, self.nx + 1), dtype=self.dtype, device=U.device)
        Fy = torch.empty((6, self.ny + 1, self.nx), dtype=self.dtype, device=U.device) if self.ny > 1 else None
        _check(lib().csh_fluxes(self._h, float(dt), _dev(U, self.dtype, self.n), _dev(Fx, self.dtype),
                                _dev(Fy, self.dtype) if Fy is not None else None))
        if self.ny == 1:
            return Fx.reshape(6, self.nx + 1), None
        return Fx, Fy

    def run_cfl(self, nsteps: int, cfl: float = 0.8, t_end: float = 0.0, U: torch.Tensor | None = None,
                work: torch.Tensor | None = None, dt_log: torch.Tensor | None = None) -> torch.Tensor:
        """Advance ``U`` (default: ``self.U``) in place by ``nsteps`` device-timed CFL steps;
        returns the per-step timesteps (GPU float64 tensor)."""
        U = self.U if U is None else U
        if work is None:
            work = getattr(self, "_work", None)
            if work is None or work.shape != U.shape or work.dtype != U.dtype:
                work = self._work = torch.empty_like(U)
        if dt_log is None:
            dt_log = torch.empty(max(nsteps, 1), dtype=torch.float64, device=U.device)
        _check(lib().csh_run_cfl(self._h, int(nsteps), float(cfl), float(t_end), _dev(U, self.dtype, self.n),
                                 _dev(work, self.dtype, self.n), _dev(dt_log, torch.float64, nsteps, True)))
        return dt_log[:nsteps]

    def run_cfl_states(self, nsteps: int, cfl: float = 0.8, U0: torch.Tensor | None = None,
                       states: torch.Tensor | None = None, dt_log: torch.Tensor | None = None):
        """``nsteps`` device-timed CFL steps from ``U0`` (default ``self.U``, left
        unchanged) keeping every state; returns (states [nsteps, *U0.shape],
        per-step timesteps as a GPU float64 tensor)."""
        U0 = self.U if U0 is None else U0
        if states is None:
            states = torch.empty((max(nsteps, 1),) + tuple(U0.shape), dtype=U0.dtype, device=U0.device)
        if dt_log is None:
            dt_log = torch.empty(max(nsteps, 1), dtype=torch.float64, device=U0.device)
        _check(lib().csh_run_cfl_states(self._h, int(nsteps), float(cfl), _dev(U0, self.dtype, self.n),
                                        _dev(states, self.dtype, nsteps * self.n, True),
                                        _dev(dt_log, torch.float64, nsteps, True)))
        return states[:nsteps], dt_log[:nsteps]

    def run_dts(self, dts: torch.Tensor, U: torch.Tensor | None = None, work: torch.Tensor | None = None):
        """Advance ``U`` (default ``self.U``) in place with the timesteps ``dts`` (GPU float64)."""
        U = self.U if U is None else U
        if work is None:
            work = getattr(self, "_work", None)
            if work is None or work.shape != U.shape or work.dtype != U.dtype:
                work = self._work = torch.empty_like(U)
        _check(lib().csh_run_dts(self._h, int(dts.numel()), _dev(dts, torch.float64), _dev(U, self.dtype, self.n),
                                 _dev(work, self.dtype, self.n)))
        return U

    def adjoint_step(self, dt: float, U: torch.Tensor, lam_next: torch.Tensor,
                     out: torch.Tensor | None = None) -> torch.Tensor:
        out = torch.empty_like(lam_next) if out is None else out
        _check(lib().csh_adjoint_step(self._h, float(dt), _dev(U, self.dtype, self.n),
                                      _dev(lam_next, self.dtype, self.n), _dev(out, self.dtype, self.n)))
        return out


    def init_state_adjoint(self, W: torch.Tensor, lam_U: torch.Tensor,
                           out: torch.Tensor | None = None) -> torch.Tensor:
        out = torch.empty_like(lam_U) if out is None else out
        _check(lib().csh_init_state_adjoint(self._h, _dev(W, self.dtype, self.n), _dev(lam_U, self.dtype, self.n),
                                            _dev(out, self.dtype, self.n)))
        return out


def _check3(code: int):
    if code != CSH_OK:
        msg = lib().csh3_last_error().decode(errors="replace")
        if code == CSH_ERR_NONPHYSICAL:
            raise NonPhysicalState(code, msg)
        raise CshError(code, msg)


class Grid3:
    """A 3-D handle (``csh3_grid``) plus the conserved state ``U`` [10, nz, ny, nx].

    ``W``: primitive fields (rho, u, v, w, Pxx, Pxy, Pxz, Pyy, Pyz, Pzz) as a
    contiguous float64 GPU tensor [10, nz, ny, nx]; ``h`` = (dx, dy, dz).
    """

    def __init__(self, W: torch.Tensor, h, bc=(BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)):
        if W.dim() != 4 or W.shape[0] != 10:
            raise ValueError("W must be [10, nz, ny, nx]")
        self.nz, self.ny, self.nx = (int(x) for x in W.shape[1:])
        self.h = tuple(float(x) for x in h)
        self.U = torch.empty_like(W)
        self.n = 10 * self.nx * self.ny * self.nz  # elements of a state
        self._h = _vp()
        _check3(lib().csh3_init_state(ctypes.byref(self._h), self.nx, self.ny, self.nz, *self.h, int(bc[0]),
                                      int(bc[1]), int(bc[2]), _dev(W, torch.float64),
                                      _dev(self.U, torch.float64), _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.csh3_destroy(h)
            self._h = None

    def step(self, dt: float, U: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
        U = self.U if U is None else U
        out = torch.empty_like(U) if out is None else out
        _check3(lib().csh3_step(self._h, float(dt), _dev(U, torch.float64, self.n), _dev(out, torch.float64, self.n)))
        return out

    def max_signal_speed(self, U: torch.Tensor | None = None) -> float:
        U = self.U if U is None else U
        s = ctypes.c_double()
        _check3(lib().csh3_max_signal_speed(self._h, _dev(U, torch.float64, self.n), ctypes.byref(s)))
        return s.value

    def last_signal_speed(self) -> float:
        s = ctypes.c_double()
        _check3(lib().csh3_last_signal_speed(self._h, ctypes.byref(s)))
        return s.value

    def run_cfl(self, nsteps: int, cfl: float = 0.8) -> torch.Tensor:
        """Advance ``self.U`` in place by ``nsteps`` device-timed steps; returns the timesteps."""
        work = getattr(self, "_work", None)
        if work is None:
            work = self._work = torch.empty_like(self.U)
        log = getattr(self, "_log", None)
        if log is None or log.numel() < max(nsteps, 1):
            log = self._log = torch.empty(max(nsteps, 1), dtype=torch.float64, device=self.U.device)
        _check3(lib().csh3_run_cfl(self._h, int(nsteps), float(cfl), _dev(self.U, torch.float64),
                                   _dev(work, torch.float64), _dev(log, torch.float64)))
        return log[:nsteps]


def init_state(W: torch.Tensor, dx: float, dy: float = 1.0, bc=(BC_PERIODIC, BC_PERIODIC)) -> Grid:
    """``csh_init_state``: a grid handle with the conserved state of ``W``."""
    return Grid(W, dx, dy, bc)


class Batch:
    """Many independent 1-D tubes (``csh_batch``): tube k holds cells
    offsets[k]:offsets[k+1] of the concatenated fields ``W`` [6, N]."""

    def __init__(self, W: torch.Tensor, offsets):
        import numpy as np
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.ntubes = int(self.offsets.size - 1)
        if self.ntubes >= 1 and W.numel() != 6 * int(self.offsets[-1]):
            raise ValueError(f"W must hold 6 x offsets[-1] = {6 * int(self.offsets[-1])} elements")
        self.U = torch.empty_like(W)
        self._work = torch.empty_like(W)
        self._h = _vp()
        _check(lib().csh_batch_init(ctypes.byref(self._h), self.ntubes,
                                    self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), F64,
                                    _dev(W, torch.float64), _dev(self.U, torch.float64), _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.csh_batch_destroy(h)
            self._h = None

    def run(self, nsteps: int, cfl: float = 0.8, threads: int = 0, dt_out: torch.Tensor | None = None):
        if dt_out is None:
            dt_out = torch.empty((self.ntubes, max(nsteps, 1)), dtype=torch.float64, device=self.U.device)
        _check(lib().csh_batch_run(self._h, int(nsteps), float(cfl), _dev(self.U, torch.float64),
                                   _dev(self._work, torch.float64),
                                   _dev(dt_out, torch.float64, self.ntubes * nsteps, True), int(threads)))
        return dt_out

    def check(self):
        """Synchronise; raise NonPhysicalState if a step of an earlier run produced a
        non-physical state (run() itself is asynchronous)."""
        _check(lib().csh_batch_status(self._h))

    def autotune(self, probe_steps: int = 8, cfl: float = 0.8) -> int:
        best = ctypes.c_int()
        _check(lib().csh_batch_autotune(self._h, int(probe_steps), float(cfl), _dev(self.U, torch.float64),
                                        ctypes.byref(best)))
        return best.value


def batch_init(W: torch.Tensor, offsets) -> Batch:
    return Batch(W, offsets)

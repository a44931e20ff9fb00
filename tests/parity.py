"""Comparison helpers shared by the GPU parity tests (no arithmetic of the scheme)."""
import numpy as np

POSITIVE = (0, 3, 5)          # rho, Exx, Eyy: positive fields
SIGNED = (1, 2, 4)            # rho u, rho v, Exy: change sign


def max_rel_error(gpu: np.ndarray, ref: np.ndarray) -> float:
    """Max relative error per field, worst over the six fields.

    Positive fields: max |g - o| / |o| cell by cell.  Sign-changing fields:
    max |g - o| / max |o| over the field; a field the reference holds at
    exactly zero everywhere is measured against the largest momentum magnitude.
    """
    g = np.asarray(gpu, dtype=np.float64).reshape(6, -1)
    o = np.asarray(ref, dtype=np.float64).reshape(6, -1)
    mom = max(np.abs(o[1]).max(), np.abs(o[2]).max(), 1e-300)
    worst = 0.0
    for m in range(6):
        d = np.abs(g[m] - o[m])
        if m in POSITIVE:
            e = (d / np.abs(o[m])).max()
        else:
            scale = np.abs(o[m]).max()
            e = d.max() / (scale if scale > 0 else mom)
        worst = max(worst, float(e))
    return worst


def field_errors(gpu: np.ndarray, ref: np.ndarray) -> list:
    g = np.asarray(gpu, dtype=np.float64).reshape(6, -1)
    o = np.asarray(ref, dtype=np.float64).reshape(6, -1)
    return [max_rel_error(np.stack([g[m]] * 6), np.stack([o[m]] * 6)) if m in POSITIVE else
            float(np.abs(g[m] - o[m]).max() / max(np.abs(o[m]).max(), 1e-300)) for m in range(6)]

"""The binding's argument checks: a buffer whose size does not match the
handle's grid is refused before any kernel sees its pointer (the kernels
index buffers from the handle's sizes alone)."""
import numpy as np
import pytest
import torch

import workloads as wl
import paper_1210_5246_amd as csh

pytestmark = pytest.mark.gpu
DEV = "cuda"


def grid(n=64):
    w = wl.periodic(n, 31)
    return csh.Grid(torch.from_numpy(w.W).to(DEV), w.dx, w.dy, (w.bcx, w.bcy))


def test_wrong_sized_states_are_refused():
    g = grid()
    small = torch.empty((6, 63, 64), dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        g.step(1e-3, small)
    with pytest.raises(ValueError):
        g.step(1e-3, g.U, small)
    with pytest.raises(ValueError):
        g.max_signal_speed(small)
    with pytest.raises(ValueError):
        g.adjoint_step(1e-3, g.U, small)
    with pytest.raises(ValueError):
        g.run_cfl(4, 0.8, dt_log=torch.empty(3, dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError):
        g.step(1e-3, g.U.float())
    # the handle still works afterwards
    out = g.step(1e-4)
    assert torch.isfinite(out).all()


def test_wrong_sized_3d_state_is_refused():
    w = wl.periodic3(8, 8, 8, seed=32)
    g = csh.Grid3(torch.from_numpy(w.W).to(DEV), (1 / 8, 1 / 8, 1 / 8))
    with pytest.raises(ValueError):
        g.step(1e-3, torch.empty((10, 8, 8, 7), dtype=torch.float64, device=DEV))


def test_batch_fields_must_match_offsets():
    t = wl.tubes(4, 5, nmin=16, nmax=32)
    W = torch.from_numpy(np.ascontiguousarray(t.W[:, :-1])).to(DEV)
    with pytest.raises(ValueError):
        csh.Batch(W, t.offsets)

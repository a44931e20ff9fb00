"""The allocation-free entry point (csh_fourier_amplitudes_noalloc) through the
C ABI: the same amplitudes as csh_fourier_amplitudes, on two calls in a row
(the second on a smaller grid and with fewer modes, so stale partial sums of
the first call would show), with no allocation inside the call."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as wl
import paper_1210_5246_amd as csh

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, flush=True)


def disc_grid(n, dtype=torch.float64):
    w = wl.disc(n, 3, 1)
    g = csh.Grid(torch.from_numpy(w.W).to(DEV, dtype), w.dx, w.dy, (w.bcx, w.bcy))
    return w, g


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_allocating_entry_point_twice(dtype):
    L = csh.lib()
    cases = [(512, 8, float("inf"), float("inf")), (200, 3, 0.3, 0.25)]   # second: smaller grid, fewer modes
    for n, m, X, Y in cases:
        w, g = disc_grid(n, dtype)
        say("noalloc fourier", n, m, X, Y, dtype)
        ref = g.fourier_amplitudes(w.x0, w.y0, m, X, Y)          # allocating entry point (host output)
        A = torch.full((m,), float("nan"), dtype=torch.float64, device=DEV)
        torch.cuda.synchronize()
        before, free_before = torch.cuda.memory_allocated(), torch.cuda.mem_get_info()[0]
        code = L.csh_fourier_amplitudes_noalloc(g._h, g.U.data_ptr(), w.x0, w.y0, X, Y, m, A.data_ptr())
        assert code == csh.CSH_OK, L.csh_last_error()
        torch.cuda.synchronize()
        # neither torch's allocator nor the device's free memory moved
        assert torch.cuda.memory_allocated() == before
        assert torch.cuda.mem_get_info()[0] == free_before
        got = A.cpu().numpy()
        # the same kernels and the same fixed summation order: bitwise equal
        assert np.array_equal(got, np.array(ref)), (got, ref)


def test_noalloc_rejects_sizes_beyond_its_limit():
    L = csh.lib()
    w, g = disc_grid(64)
    A = torch.zeros(32, dtype=torch.float64, device=DEV)
    assert L.csh_fourier_amplitudes_noalloc(g._h, g.U.data_ptr(), w.x0, w.y0, 1.0, 1.0, 17, A.data_ptr()) == \
        csh.CSH_ERR_ARG
    assert b"CSH_FOURIER_MAX_M" in L.csh_last_error()
    assert L.csh_fourier_amplitudes_noalloc(g._h, g.U.data_ptr(), w.x0, w.y0, 1.0, 1.0, 0, A.data_ptr()) == \
        csh.CSH_ERR_ARG
    assert L.csh_fourier_amplitudes_noalloc(g._h, g.U.data_ptr(), w.x0, w.y0, 1.0, 1.0, 4, None) == csh.CSH_ERR_ARG

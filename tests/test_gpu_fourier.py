"""The GPU global Fourier amplitudes (Sec. 4.4) against the oracle's.

Amplitudes are normalised by the disc mass, so 1 is their natural scale (a
point mass has A_m = 1).  The two sides add 10^4..10^7 terms in different
orders and form exp(i m phi) differently (powers of (x + i y) / R against
cos / sin of atan2); the rounding of such a sum is ~1e-16 of the sum of the
terms' magnitudes, i.e. of the mass: the bar is |A_gpu - A_oracle| <= 1e-13
absolute, and 1e-12 relative where A_m > 1e-3 (a small amplitude is itself a
near-cancellation, which no relative bound survives).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as wl
import paper_1210_5246_amd as csh

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ogrid(w):
    return oracle.Grid(w.nx, w.ny, w.dx, w.dy, w.bcx, w.bcy, w.x0, w.y0, w.vc, w.rc)


def gpu_grid(w, dtype=torch.float64):
    return csh.Grid(torch.from_numpy(np.ascontiguousarray(w.W)).to(DEV, dtype), w.dx, w.dy, (w.bcx, w.bcy))


def close(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    assert np.abs(got - ref).max() <= 1e-13, np.abs(got - ref).max()
    big = ref > 1e-3
    assert np.all(np.abs(got[big] - ref[big]) <= 1e-12 * ref[big])


@pytest.mark.parametrize("n", [256, 255])
def test_disc_whole_grid(n):
    w = wl.disc(n, 3, 1)
    say("fourier disc", n)
    g = gpu_grid(w)
    ref = oracle.fourier_amplitudes(ogrid(w), oracle.cons_field(w.W), 16)
    got = g.fourier_amplitudes(w.x0, w.y0, 16)
    close(got, ref)
    assert ref[1] > 1e-3                          # the seeded two-armed perturbation
    assert got == g.fourier_amplitudes(w.x0, w.y0, 16)   # fixed summation order


@pytest.mark.parametrize("region", [(0.2, 0.2), (0.31, 0.07), (0.01, 0.5)])
def test_region_and_ragged_offset_grid(region):
    w = wl.periodic(130, 51)
    w.W = np.ascontiguousarray(w.W[:, :97, :130])
    w.nx, w.ny, w.dx, w.dy = 130, 97, 0.9 / 130, 0.8 / 97
    w.x0, w.y0 = -0.37, -0.52
    say("fourier region", region)
    g = gpu_grid(w)
    X, Y = region
    ref = oracle.fourier_amplitudes(ogrid(w), oracle.cons_field(w.W), 7, X, Y)
    close(g.fourier_amplitudes(w.x0, w.y0, 7, X, Y), ref)


def test_point_mass_and_origin_cell():
    say("fourier point masses")
    n = 65                                          # odd: the centre cell sits on the origin
    w = wl.periodic(n, 52)
    w.W[0] = 1e-300
    w.W[0, 32, 32] = 1.0                            # on the origin: no angle
    w.W[0, 10, 50] = 2.0
    w.x0 = w.y0 = -0.5
    w.dx = w.dy = 1.0 / n
    g = gpu_grid(w)
    got = np.array(g.fourier_amplitudes(w.x0, w.y0, 5))
    np.testing.assert_allclose(got, 2.0 / 3.0, rtol=1e-13)


def test_after_fifty_steps_matches_oracle_on_the_same_state():
    w = wl.disc(512, 3, 50)
    say("fourier after 50 steps at 512^2")
    g = gpu_grid(w)
    g.set_potential(w.vc, w.rc, w.x0, w.y0)
    A0 = np.array(g.fourier_amplitudes(w.x0, w.y0, 6))
    g.run_cfl(50, 0.8)
    got = g.fourier_amplitudes(w.x0, w.y0, 6)
    close(got, oracle.fourier_amplitudes(ogrid(w), g.U.cpu().numpy(), 6))
    say("A_m before / after:", A0, np.array(got))


def test_disc_4096_full_size():
    w = wl.disc(4096, 3, 1)
    say("fourier disc 4096^2 (oracle first)")
    ref = oracle.fourier_amplitudes(ogrid(w), oracle.cons_field(w.W), 16)
    g = gpu_grid(w)
    close(g.fourier_amplitudes(w.x0, w.y0, 16), ref)


def test_fp32_state():
    w = wl.disc(256, 3, 1)
    say("fourier fp32")
    g = gpu_grid(w, torch.float32)
    U32 = g.U.double().cpu().numpy()              # the FP32 state, exactly
    ref = oracle.fourier_amplitudes(ogrid(w), U32, 6)
    close(g.fourier_amplitudes(w.x0, w.y0, 6), ref)


def test_argument_errors():
    say("fourier argument errors")
    w = wl.disc(64, 3, 1)
    g = gpu_grid(w)
    for kw in ({"m_max": 0}, {"m_max": 17}, {"X": 0.0}, {"Y": -1.0}):
        with pytest.raises(csh.CshError):
            g.fourier_amplitudes(w.x0, w.y0, **kw)
    t = wl.sod(64)
    g1 = csh.Grid(torch.from_numpy(t.W).to(DEV), t.dx, 1.0, (t.bcx, t.bcy))
    with pytest.raises(csh.CshError):
        g1.fourier_amplitudes(0.0, 0.0, 4)

"""Batched 1-D tubes (one persistent, graph-replayed launch) against the
oracle run tube by tube, and against the plain one-grid-per-launch path."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as wl
import paper_1210_5246_amd as csh
from parity import max_rel_error

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def subset(t, ks):
    """A Tubes object holding tubes ks of t."""
    lengths = t.lengths[ks]
    offsets = np.zeros(len(ks) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    W = np.concatenate([t.W[:, t.offsets[k]:t.offsets[k + 1]] for k in ks], axis=1)
    return wl.Tubes(lengths, offsets, np.ascontiguousarray(W), t.left[ks], t.right[ks], t.cfl, t.nsteps)


def oracle_tube(t, k, nsteps):
    n = int(t.lengths[k])
    g = oracle.Grid(n, 1, 1.0 / n, 1.0, oracle.BC_OUTFLOW, oracle.BC_OUTFLOW)
    W = np.ascontiguousarray(t.W[:, t.offsets[k]:t.offsets[k + 1]])
    return oracle.run_cfl(g, oracle.cons_field(W), nsteps=nsteps, cfl=t.cfl)


@pytest.mark.parametrize("threads", [64, 256, 1024])
def test_batch_matches_oracle(threads):
    full = wl.tubes()
    ks = [0, 1, 2, 3, 4, 5, int(np.argmax(full.lengths)), int(np.argmin(full.lengths))]
    t = subset(full, ks)
    nsteps = 200
    say("batch vs oracle, threads", threads, "lengths", t.lengths.tolist())
    b = csh.Batch(torch.from_numpy(t.W).to(DEV), t.offsets)
    dts = b.run(nsteps, t.cfl, threads=threads).cpu().numpy()
    U = b.U.cpu().numpy()
    for j in range(len(ks)):
        ref, dts_o = oracle_tube(t, j, nsteps)
        np.testing.assert_allclose(dts[j], dts_o, rtol=1e-12)
        got = U[:, t.offsets[j]:t.offsets[j + 1]]
        assert max_rel_error(got, ref) <= 1e-10, (j, t.lengths[j])


@pytest.mark.parametrize("threads", [None, 1024])
def test_full_batch_sampled_tubes_match_oracle(threads):
    """The benchmark's batch and launch: all 512 tubes in one persistent
    launch (the autotuner's workgroup size, and 1024), 200 steps; sampled
    tubes (the longest, the shortest and ten at random) against the oracle
    run tube by tube, timesteps to 1e-12 and states to 1e-10."""
    t = wl.tubes()
    nsteps = 200
    b = csh.Batch(torch.from_numpy(t.W).to(DEV), t.offsets)
    if threads is None:
        threads = b.autotune(probe_steps=8)
        b = csh.Batch(torch.from_numpy(t.W).to(DEV), t.offsets)  # a fresh handle and state
    say("full batch vs oracle on sampled tubes, threads", threads)
    dts = b.run(nsteps, t.cfl, threads=threads).cpu().numpy()
    U = b.U.cpu().numpy()
    r = np.random.default_rng(41)
    ks = sorted({int(np.argmax(t.lengths)), int(np.argmin(t.lengths))} | set(r.choice(512, 10, replace=False).tolist()))
    for k in ks:
        ref, dts_o = oracle_tube(t, k, nsteps)
        np.testing.assert_allclose(dts[k], dts_o, rtol=1e-12)
        got = U[:, t.offsets[k]:t.offsets[k + 1]]
        assert max_rel_error(got, ref) <= 1e-10, (k, t.lengths[k])


def test_batch_edge_lengths_and_odd_steps():
    lengths = np.array([1, 2, 3, 5, 59, 60, 61, 121, 4096], dtype=np.int64)
    r = np.random.default_rng(40)
    offsets = np.zeros(lengths.size + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    W = np.zeros((6, int(offsets[-1])))
    for k, n in enumerate(lengths):
        sl = slice(int(offsets[k]), int(offsets[k + 1]))
        x = (np.arange(n) + 0.5) / n
        W[0, sl] = 0.6 + 0.3 * np.sin(2 * np.pi * x + k)
        # phases keep every field away from exact cancellation on 1-3 cell tubes
        W[1, sl] = 0.2 * np.cos(2 * np.pi * x + 0.7)
        W[2, sl] = 0.1
        W[3, sl] = 0.5 + 0.2 * np.cos(4 * np.pi * x + 0.3)
        W[4, sl] = 0.05 * np.sin(2 * np.pi * x + 0.4)
        W[5, sl] = 0.4
    t = wl.Tubes(lengths, offsets, W, np.zeros((9, 4)), np.zeros((9, 4)))
    nsteps = 7
    say("batch edge lengths, odd steps")
    b = csh.Batch(torch.from_numpy(W).to(DEV), offsets)
    b.run(nsteps, 0.8, threads=128)
    U = b.U.cpu().numpy()
    for k in range(lengths.size):
        ref, _ = oracle_tube(t, k, nsteps)
        assert max_rel_error(U[:, offsets[k]:offsets[k + 1]], ref) <= 1e-11, int(lengths[k])


def test_thread_counts_agree_bitwise_and_autotune(monkeypatch):
    monkeypatch.setenv("CSH_TUNE_CACHE", "off")   # probe, whatever a cache holds
    t = wl.tubes(ntubes=64, seed=41)
    say("thread counts bitwise, autotune")
    W = torch.from_numpy(t.W).to(DEV)
    outs = []
    for th in (64, 128, 256, 512, 1024):
        b = csh.Batch(W, t.offsets)
        d = b.run(20, 0.8, threads=th)
        outs.append((b.U.clone(), d.clone()))
    for U, d in outs[1:]:
        assert torch.equal(U, outs[0][0]) and torch.equal(d, outs[0][1])
    b = csh.Batch(W, t.offsets)
    U0 = b.U.clone()
    best = b.autotune(probe_steps=4)
    assert best in (64, 128, 256, 512, 1024)
    assert torch.equal(b.U, U0)          # tuning works on scratch copies
    b.run(20, 0.8)                        # default = tuned size
    assert torch.equal(b.U, outs[0][0])


def test_autotune_persists_its_choice(tmp_path, monkeypatch):
    """The tuned workgroup size is recorded per batch shape and device kind;
    a later handle of the same shape takes the record without probing."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("CSH_TUNE_CACHE", str(cache))
    t = wl.tubes(ntubes=64, seed=41)
    say("autotune cache")
    W = torch.from_numpy(t.W).to(DEV)
    best = csh.Batch(W, t.offsets).autotune(probe_steps=4)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    key, th = lines[0].rsplit(" ", 1)
    assert int(th) == best
    props = torch.cuda.get_device_properties(0)
    assert f"cus={props.multi_processor_count};" in key and ";tubes=64;" in key
    assert f";cells={int(t.offsets[-1])};" in key and key.endswith(f";maxlen={int(t.lengths.max())}")
    # a record for this key that the probe need not pick is taken as it stands
    other = 64 if best != 64 else 128
    cache.write_text(f"{key} {other}\n")
    assert csh.Batch(W, t.offsets).autotune(probe_steps=4) == other
    assert cache.read_text().splitlines() == [f"{key} {other}"]   # a hit records nothing
    # another shape misses and is recorded beside it
    t2 = subset(t, list(range(10)))
    best2 = csh.Batch(torch.from_numpy(t2.W).to(DEV), t2.offsets).autotune(probe_steps=4)
    assert cache.read_text().splitlines()[1].endswith(f" {best2}")
    # switched off: probes, records nothing
    monkeypatch.setenv("CSH_TUNE_CACHE", "off")
    assert csh.Batch(W, t.offsets).autotune(probe_steps=4) in (64, 128, 256, 512, 1024)
    assert len(cache.read_text().splitlines()) == 2


def test_batch_equals_plain_path_per_tube():
    """The plain path: for each tube its own grid, and per step a host round
    trip for the timestep (max_signal_speed) and one launch (step)."""
    full = wl.tubes()
    ks = list(range(0, 512, 32))
    t = subset(full, ks)
    nsteps = 200
    say("batch vs plain per-tube path", len(ks), "tubes")
    b = csh.Batch(torch.from_numpy(t.W).to(DEV), t.offsets)
    dts = b.run(nsteps, 0.8).cpu().numpy()
    U = b.U.cpu().numpy()
    for j in range(len(ks)):
        W = torch.from_numpy(np.ascontiguousarray(t.W[:, t.offsets[j]:t.offsets[j + 1]])).to(DEV)
        n = int(t.lengths[j])
        g = csh.Grid(W, 1.0 / n, 1.0, (csh.BC_OUTFLOW, csh.BC_OUTFLOW))
        Ug = g.U
        for s in range(nsteps):
            dt = 0.8 / g.max_signal_speed(Ug)
            assert dt == pytest.approx(dts[j, s], rel=1e-14)
            Ug = g.step(dt, Ug)
        got = U[:, t.offsets[j]:t.offsets[j + 1]]
        assert max_rel_error(got, Ug.cpu().numpy()) <= 1e-12


def test_batch_status_reports_a_nonphysical_tube():
    """run() is asynchronous and checks every new state on the device;
    check() reports a tube that went non-physical (here a negative density
    slipped into one tube between runs) and passes on a clean batch."""
    t = subset(wl.tubes(), [0, 1, 2, 3])
    say("batch status, lengths", t.lengths.tolist())
    b = csh.Batch(torch.from_numpy(t.W).to(DEV), t.offsets)
    b.run(5, t.cfl)
    b.check()
    c = int(t.offsets[2]) + int(t.lengths[2]) // 2
    b.U[0, c] = -b.U[0, c]
    b.run(1, t.cfl)
    with pytest.raises(csh.NonPhysicalState):
        b.check()

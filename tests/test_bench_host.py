"""Host logic of bench.py (no GPU): the one-GPU guard, the committed counter
summary and its source-hash guard, and the arithmetic of the VALU figures."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_committed_counters_match_the_kernel_sources():
    t = bench.measured_counters(4096)
    assert t, "profiles/sweep_disc4096_f64_traffic.json was taken on other kernel sources"
    assert t["kernel_source_hash"] == bench.sweep_source_hash()
    alg = 96 * 4096 * 4096
    assert t["algorithmic_bytes_per_launch"] == alg
    assert 1.0 <= t["bytes_per_launch"] / alg < 1.5


def test_counters_are_dropped_when_the_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: "0" * 16)
    assert bench.measured_counters(4096) == {}


def test_valu_summary_arithmetic():
    cells = 1000
    t = {"valu": {"fp64_flops_per_launch": 2.0e6, "valu_busy": 0.9, "valu_lane_instructions_per_cell": 500.0,
                  "fp64_flops_per_cell": 2000.0}}
    v = bench.valu_summary(t, 1e-6, cells)
    assert v["fp64_tflops"] == pytest.approx(2.0)
    assert v["fp64_frac"] == pytest.approx(2.0 / 78.6)
    assert v["issue_tlane_instr_per_s"] == pytest.approx(0.5)
    assert v["issue_peak_tlane_instr_per_s"] == pytest.approx(256 * 4 * 16 * 2.4e9 / 1e12)
    assert bench.valu_summary({}, 1e-6, cells) is None


def test_cpu_model_is_a_name():
    name = bench.cpu_model()
    assert isinstance(name, str) and name

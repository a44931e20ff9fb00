"""The benchmark's output contract on a GPU: one JSON line on stdout with the
headline fields, the roofline block and the workload named in `config`
(a short run of the disc at 512^2 with the other legs switched off)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line_with_the_contract_fields():
    print("bench.py --n 512 --steps 2 --warmup 1 (one leg)", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--n", "512", "--steps", "2", "--warmup", "1",
                        "--no-cpu", "--no-batch", "--no-adjoint", "--no-fp32", "--no-kt", "--no-fourier", "--no-hllc",
                        "--no-3d"], capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [x for x in r.stdout.splitlines() if x.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["dtype"] == "f64" and d["unit"] == "cell-updates/s"
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert d["value"] == pytest.approx(2 * 512 * 512 / (d["ms_per_step"] * 2 / 1e3), rel=1e-9)
    assert "workload" in d["config"] and "model" not in d["config"]
    rf = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"])
    assert rf["traffic"] is None          # the committed counters are of the 4096^2 disc

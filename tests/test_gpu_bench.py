"""bench.py on the GPU, briefly: it prints one JSON line with the fields the
benchmark record needs (metric, throughput, step count, dtype, workload,
roofline of the dominant kernel), and its throughput agrees with its own
milliseconds per step (4 field evaluations per RK4 step)."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line():
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "20", "--warmup", "3",
                        "--no-cpu", "--no-extras", "--no-b2b"],
                       capture_output=True, text=True, timeout=110, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert (d["n_gpus"], d["steps"], d["warmup"], d["unit"], d["dtype"]) == (1, 20, 3, "evals/s", "f32")
    assert d["higher_is_better"] is True and d["cpu_baseline"] is None
    assert "workload" in d["config"] and "model" not in d["config"]
    assert d["value"] == pytest.approx(4 * 1e3 / d["ms_per_step"], rel=1e-9)
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert 0 < rf["frac"] < 1 and rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], rel=1e-9)

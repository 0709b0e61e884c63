"""bench.py's output contract on a GPU: one JSON line with the throughput, the roofline of the
dominant kernel and the error against the oracle golden, here on the small named shapes (config 1)
with a short run."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line_with_the_contract_keys():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--config", "1", "--batch", "32", "--steps", "2",
           "--warmup", "1", "--no-cpu-baseline", "--no-extras", "--serving-seconds", "0"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=280)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["unit"] == "sets/s" and d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["dtype"] == "f16x3" and d["cpu_baseline"] is None
    assert d["value"] == pytest.approx(32 / (d["ms_per_step"] * 1e-3), rel=1e-6)
    assert "workload" in d["config"] and d["config"]["batch"] == 32
    roof = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert roof["bound"] in ("hbm", "mfma") and 0 < roof["frac"] < 1
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], rel=1e-9)
    step = roof["step"]  # the whole step against HBM: at least the dominant kernel's bytes, in more time
    assert step["algorithmic_bytes"] >= roof["algorithmic_bytes"] and 0 < step["frac"] < 1
    assert step["frac"] == pytest.approx(step["achieved"] / step["peak"], rel=1e-9)
    print("config 1 bench:", d["value"], "sets/s, error", d.get("max_rel_err_vs_oracle"), flush=True)
    assert d["max_rel_err_vs_oracle"] <= 1e-3

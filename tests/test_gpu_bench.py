"""bench.py's output contract on a GPU, at a small size: exactly one JSON line
on stdout with the fields the benchmark line promises (value and
ms_per_step consistent, the roofline object of the dominant kernel, the
oracle CPU baseline).  The benchmark runs as a child process."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line_contract():
    systems = 3
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--N", "32", "--systems", str(systems),
           "--steps", "1", "--warmup", "1", "--no-large", "--cpu-iters", "3"]
    print("running", " ".join(cmd[2:]), flush=True)
    r = subprocess.run(cmd, cwd=ROOT, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 1
    assert d["higher_is_better"] is False and d["unit"] == "s/system" and d["dtype"] == "f64"
    assert d["value"] > 0 and d["ms_per_step"] == pytest.approx(d["value"] * systems * 1e3, rel=1e-9)
    assert "workload" in d["config"] and d["config"]["n"] == 32 ** 3
    rl = d["roofline"]
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert rl["achieved"] > 0 and rl["frac"] == pytest.approx(rl["achieved"] / rl["peak"])
    # the committed counter summary covers the 128^3 workload only
    assert rl["traffic"] is None
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == "s/system" and cb["cores"] >= 1 and cb["value"] > 0
    assert isinstance(cb["sample"], str) and cb["sample"]
    # every solve of the sequences met the tolerance
    assert d["true_relres_max"] <= 1.01e-8 and d["mixed_true_relres_max"] <= 1e-8

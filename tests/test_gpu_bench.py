"""bench.py's output contract, on a small cavity.

- One JSON line on stdout with the fields the benchmark record needs; `value` is
  cells x steps over the event-timed region, and `ms_per_step` agrees with it.
- The roofline object follows from the dominant kernel's average launch time
  (algorithmic bytes per launch over that time), and the 3-step comparison
  sweep carries the same fields.
- The settle sweeps on a twin cavity are reported (`settle`).
- `--gpus` above 1 exits with status 2 and a message before touching the GPU
  (a CPU test).
"""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, timeout=600):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=timeout, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"], timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.gpu
def test_bench_line_contract_small_cavity():
    n, steps = 96, 16
    r = _run(["--n", str(n), "--steps", str(steps), "--warmup", "4", "--no-serving", "--cpu-steps", "1",
              "--cpu-steps-1thread", "1", "--numpy-steps", "1"])
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [x for x in r.stdout.splitlines() if x.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == steps and d["warmup"] == 4
    assert d["higher_is_better"] is True and d["vs_baseline"] is None and d["dtype"] == "f32"
    assert "workload" in d["config"]
    cells = n ** 3
    assert d["value"] > 0
    # value and ms_per_step describe the same timed region
    assert abs(cells * steps / (d["ms_per_step"] * steps / 1e3) / 1e9 - d["value"]) <= 0.01 * d["value"]
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["peak"] == 8000.0 and rf["unit"] == "GB/s"
    # achieved: the algorithmic bytes of one launch of the dominant kernel over its average time
    assert rf["bytes_per_launch"] == pytest.approx(60 * cells)
    assert rf["achieved"] == pytest.approx(rf["bytes_per_launch"] / (rf["avg_launch_ms"] / 1e3) / 1e9, rel=1e-3)
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], abs=1e-4)
    assert d["config"]["steps_per_launch"] == 4 and rf["launches_timed"] == steps // 4
    assert rf["traffic"] is None  # counters are recorded for the 512^3 cavity only
    # the settle sweeps ran on a twin cavity with the same schedule, before the warm-up steps
    st = d["settle"]
    assert st["kind"].startswith("twin cavity") and st["steps"] > 0 and st["steps"] % 4 == 0
    other = d["other_schedule"]
    assert other["steps_per_launch"] == 3 and other["gcells"] > 0
    assert other["frac"] == pytest.approx(60 * cells / 1e9 / (other["avg_launch_ms"] / 1e3) / 8000.0, abs=1e-4)
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["unit"] == "Gcell-updates/s"

"""GPU: the bench's JSON line carries the fields its contract names, with the parity
condition of the metric met (256 x 256 x 128 workload, a few timed steps); the adjoint
bench's line with two shots in one solver."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(600)
def test_bench_line_fields():
    print("bench.py --workload c2 --steps 3 --warmup 1 --cpu-budget 1 --no-equal-accuracy", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "c2", "--steps", "3",
                        "--warmup", "1", "--cpu-budget", "1", "--no-equal-accuracy"],
                       capture_output=True, text=True, timeout=580, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["higher_is_better"] is True
    assert d["unit"] == "DOF-updates/s" and d["data"] == "synthetic" and d["vs_baseline"] is None
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert "256x256x128" in d["config"]["workload"] and d["config"]["path"] == "int8"
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12
    # the roofline's bytes per launch over the measured time give the reported rate
    assert abs(rf["achieved"] * 1e9 - rf["algorithmic_bytes_per_launch"] / (d["ms_per_step"] * 1e-3)) < 1e-6 * rf[
        "achieved"] * 1e9
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == "DOF-updates/s" and cb["cores"] >= 1 and cb["value"] > 0
    assert cb["sample"]
    # the metric's accuracy condition, over the whole run whatever the timed steps
    assert d["int8_vs_fp64"]["trace_rel_l2"] <= 1e-9 and d["int8_vs_fp64"]["steps_compared"] == 2000
    assert d["timed_from_step"] == 1000 and set(d["full_run_ms_per_step"]) == {"fp64", "int8", "fp64-sf"}
    assert d["int8_m6_path"]["vs_fp64"]["trace_rel_l2"] <= 1e-9


@pytest.mark.timeout(600)
def test_adjoint_bench_line_with_two_shots():
    """The 96^3 adjoint bench with two shots in one solver: one JSON line whose value is the
    whole solver's rate, and shot 0's gradient against the stored oracle adjoint."""
    print("bench.py --workload c4-adjoint --paths int8 --adjoint-shots 2 --no-autotune", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "c4-adjoint", "--paths",
                        "int8", "--adjoint-shots", "2", "--no-autotune"],
                       capture_output=True, text=True, timeout=580, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    assert d["config"]["shots"] == 2 and d["config"]["path"] == "int8" and d["steps"] == 1000
    p = d["paths"]["int8"]
    assert p["forward_ms_per_step"] > 0 and p["adjoint_ms_per_step"] == d["ms_per_step"]
    assert abs(d["value"] - p["adjoint_value"]) <= 1e-9 * d["value"]
    vo = p["vs_oracle"]
    assert vo["J"] <= 1e-9 and vo["g_lam"] <= 1e-9 and vo["g_mu"] <= 1e-9 and vo["voxels"] == 50

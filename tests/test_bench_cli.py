"""bench.py on the CPU: the one-GPU guard, the command line, and the CPU
baseline legs at small sizes (nothing here touches a GPU)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_studies():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for word in ("precision", "echo", "gue", "long", "sizes", "adjoint", "--depths", "--sweep-variant",
                 "--cpu-baseline-scaling", "--sweep-only"):
        assert word in r.stdout


def test_cpu_baseline_at_small_size():
    res = bench.cpu_baseline(12, 3)
    assert res["kind"] == "oracle" and res["unit"] == "periods/s" and res["cores"] == 1
    assert res["value"] > 0 and abs(res["value"] * res["s_per_period"] - 1.0) < 1e-9
    json.dumps(res)


def test_cpu_baseline_scaling_fit_at_small_sizes():
    res = bench.cpu_baseline_scaling([10, 12], nrep=1)
    assert [r["L"] for r in res["rows"]] == [10, 12]
    assert res["a_ns"] > 0 and res["fit_s_per_period_L30"] > 0
    json.dumps(res)


def test_traffic_is_reported_only_for_the_measured_kernel_code():
    t = bench.measured_traffic()
    if bench.kernel_code_hash() == bench.TRAFFIC["kernel_code_sha256_16"]:
        assert abs(t - 16 * 2**30) / (16 * 2**30) < 1e-3   # 16 B per amplitude per pass at L = 30
    else:
        assert t is None

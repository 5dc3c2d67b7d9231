"""Host-side checks of bench.py's command line (no GPU work)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_no_gpu_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    r = run_bench("--steps", "1", "--warmup", "0")
    assert r.returncode == 1
    assert "no GPU" in r.stderr


def test_traffic_table_names_compile_time_widths():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.KRON_TRAFFIC_BATCH == 512
    assert set(bench.KRON_TRAFFIC) <= {8, 16}
    # bytes per launch lie between the algorithmic 1.2325 GB and 5 % above it
    assert all(1.2325e9 <= v <= 1.05 * 1.2325e9 for v in bench.KRON_TRAFFIC.values())

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


def test_traffic_table_is_keyed_by_workload_and_batch():
    """Stabilisation HBM bytes are quoted only for the (workload, batch) they
    were counted on; at least the QR's own operand traffic (the pivoted copy
    of X written and read, Q written) per field."""
    sys.path.insert(0, ROOT)
    import bench
    from slq_inputs import WORKLOADS
    for (workload, batch), v in bench.STAB_TRAFFIC.items():
        m = WORKLOADS[workload]
        assert batch > 0 and v > 3 * 8 * m.n_sites ** 2 * batch

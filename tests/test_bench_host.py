"""bench.py on the host: the one-GPU contract and the counter bookkeeping (no GPU needed)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_figure_is_keyed_to_the_kernel_source():
    import bench
    assert bench.measured_traffic("no such mode") is None
    rec = bench.MEASURED_TRAFFIC["fp32_3m"]
    got = bench.measured_traffic("fp32_3m")
    # either the recorded counter figure (source unchanged since the counters) or null
    assert got is None or got == rec["bytes"]
    assert rec["bytes"] > 0 and len(rec["kernel_source_sha256"]) == 64

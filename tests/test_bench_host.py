"""bench.py host-side behaviour (no GPU): it measures one GPU only and says
so for --gpus N > 1, and it records the host cores the CPU baseline uses."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_host_cpu_record():
    import bench
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and 1 <= h["threads"] <= h["nproc"]
    json.dumps(h)

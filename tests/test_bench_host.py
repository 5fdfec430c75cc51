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


def test_multichannel_roofline_bounds():
    """The bound of each multi-channel run follows its flop/byte against the
    ridge of its peak: BF16 3x3 (192 flop/B) is HBM-bound, BF16 5x5 (532) is
    MFMA-bound, the FP32 path (144 and 400 flop/B) is ALU-bound; achieved and
    frac follow from the algorithmic bytes or flops over the time."""
    import bench
    n, side, c = 16, 128, 64
    for bf16, f, bound in ((True, 3, "hbm"), (True, 5, "mfma"), (False, 3, "alu"), (False, 5, "alu")):
        flops = 2.0 * n * side * side * c * c * f * f
        r = bench.multichannel_roofline(bf16, f, flops, 0.05)
        eb = 2 if bf16 else 4
        assert r["algorithmic_bytes"] == n * side * side * c * (eb + 4) + c * f * f * c * eb
        assert r["bound"] == bound
        if bound == "hbm":
            assert r["unit"] == "GB/s" and r["peak"] == bench.HBM_PEAK_GBS
            assert abs(r["achieved"] - r["algorithmic_bytes"] / 0.05e-3 / 1e9) < 0.1
        else:
            assert r["unit"] == "TFLOP/s"
            assert abs(r["achieved"] - flops / 0.05e-3 / 1e12) < 0.01
        assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3


def test_bench_line_is_strict_json():
    import bench
    line = json.dumps(bench.finite_or_none({"a": float("nan"), "b": [1.5, float("inf")], "c": {"d": -float("inf")}}),
                      allow_nan=False)
    assert json.loads(line) == {"a": None, "b": [1.5, None], "c": {"d": None}}

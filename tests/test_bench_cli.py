"""bench.py contract checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_flop_model_scales_with_walkers():
    sys.path.insert(0, ROOT)
    import bench
    a = bench.algorithmic_flops("slater_sample", 128, 1, 1535)
    b = bench.algorithmic_flops("slater_sample", 128, 16384, 1535)
    assert b == 16384 * a
    # the three contractions alone: 3 x 2 x (2 N NS^2) flops per walker and sample
    assert a > 3 * 2 * 2 * 128 * 64 * 64

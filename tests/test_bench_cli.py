"""bench.py's command line on the CPU: more than one GPU is refused with a
message and exit status 2 before any GPU work, and the roofline helpers
price the kernels as the library dispatches them."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_switch_pricing_follows_the_dispatch_rule():
    import bench
    # complex64 batches of >= 32 right-hand sides at q <= 9 run on the matrix cores
    assert bench.switch_on_mfma(9, 64) and bench.switch_on_mfma(3, 32)
    assert not bench.switch_on_mfma(9, 31) and not bench.switch_on_mfma(10, 64)
    # 4 q^4 N^2 flops per right-hand side: q = 9, N = 1024
    assert bench.mfma_switch_flops(1024, 9) == 4.0 * 9 ** 4 * 1024 ** 2

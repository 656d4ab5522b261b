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


def test_kernel_pricing_follows_the_dispatch_rule():
    import bench
    # complex64 chunks of >= 32 right-hand sides at q <= 9: switches on the matrix cores
    assert {"switch", "switch_adj"} <= set(bench.mfma_kinds(9, 3, 64))
    assert {"switch", "switch_adj"} <= set(bench.mfma_kinds(3, 3, 32))
    assert "switch" not in bench.mfma_kinds(9, 3, 31) and not bench.mfma_kinds(10, 3, 64)
    # initialisation on the matrix cores only at s = 3
    assert "init" in bench.mfma_kinds(9, 3, 1) and "init" not in bench.mfma_kinds(9, 2, 64)
    # levels only with contract "mfma"
    assert "plevel" not in bench.mfma_kinds(9, 3, 64)
    assert {"plevel", "xlevel_adj"} <= set(bench.mfma_kinds(9, 3, 64, "mfma"))
    # switch: 4 q^4 N^2 flops per right-hand side (q = 9, N = 1024), both halves of the weights read and written
    nbytes, flops = bench.algorithmic_work("switch", 1024, 9, 3, 1)
    assert flops == 4.0 * 9 ** 4 * 1024 ** 2 and nbytes == 2 * 1024 ** 2 * 81 * 8
    r = bench.roofline_of("switch", 1.0, 1, 1024, 9, 3, 64)
    assert r["bound"] in ("hbm", "mfma") and abs(r["frac"] - max(r["hbm_frac"], r["fp32_frac"])) < 1e-12
    # the BF16 p-level is priced against the BF16 matrix-core peak, the other kinds against FP32
    assert "plevel" in bench.mfma_kinds(7, 3, 64, "bf16") and "xlevel" not in bench.mfma_kinds(7, 3, 64, "bf16")
    rb = bench.roofline_of("plevel", 1e-3, 1, 512, 7, 3, 64, "bf16")
    rf = bench.roofline_of("plevel", 1e-3, 1, 512, 7, 3, 64, "fp")
    assert rb["compute_peak_tflops"] == bench.BF16_PEAK_TFLOPS and "compute_peak_tflops" not in rf
    if rb["bound"] != "hbm":
        assert rb["bound"] == "mfma" and rb["peak"] == bench.BF16_PEAK_TFLOPS
    assert abs(rb["fp32_frac"] * bench.BF16_PEAK_TFLOPS - rf["fp32_frac"] * bench.FP32_PEAK_TFLOPS) < 1e-6

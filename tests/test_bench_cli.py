"""bench.py's host-side contract (no GPU): it measures one GPU only and says so
when asked for more, before touching any device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr
    assert r.stdout.strip() == ""


def test_bench_roofline_constants():
    sys.path.insert(0, ROOT)
    import bench

    # non-packed FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
    assert abs(bench.PEAK_FP32_NONPACKED_TFLOPS - 78.6432) < 1e-9
    assert bench.PEAK_FP32_PUBLISHED_TFLOPS == 157.3
    # the algorithmic count of the measured evaluation: 59 flops and 3 exponentials per pair
    assert bench.FLOPS_PER_PAIR == 59
    assert bench.FLOPS_PER_PAIR == bench.FLOPS_ROW_PER_PAIR + bench.FLOPS_COL_PER_PAIR
    assert bench.EXPS_ROW_PER_PAIR + bench.EXPS_COL_PER_PAIR == 3
    # the traffic figure is either the measured one or withheld, never something else
    assert bench.k_row_traffic() in (None, bench.K_ROW_TRAFFIC_BYTES)

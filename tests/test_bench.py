"""Host logic of bench.py (no GPU): the multi-GPU refusal, the dominant kernel's rate
from the union of its launch intervals, and the counter-measured traffic that is
reported only for the LU source and launch size it was measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _stats(busy, own, launches=28, flops_per_launch=6.87194767360e11):
    return {"ms_gemm_busy": busy, "ms_gemm": own, "gemm_launches": launches,
            "gemm_flops": launches * flops_per_launch}


def test_rate_from_the_union_of_the_intervals():
    # 28 launches whose union is 10 ms each on average and whose own intervals add up
    # to 12 ms each: the rate follows the union
    r = bench.roofline(_stats(280.0, 336.0), "fp64")
    assert r["achieved"] == pytest.approx(6.87194767360e11 / 10e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    assert r["avg_launch_ms"] == pytest.approx(10.0)
    assert r["avg_launch_ms_own_interval"] == pytest.approx(12.0)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert bench.roofline(_stats(0.0, 0.0, 0), "fp32")["achieved"] == 0.0


def test_traffic_only_for_the_measured_configuration():
    fpl = 687194767360.0
    t = bench.measured_traffic("qep_n1024_16x16", "fp64", fpl)
    assert t is None or t > 0
    # another workload, precision or launch size never takes the stored figure
    assert bench.measured_traffic("qep_n64_4x4", "fp64", fpl) is None
    assert bench.measured_traffic("qep_n1024_16x16", "fp32", fpl) is None
    assert bench.measured_traffic("qep_n1024_16x16", "fp64", 0.5 * fpl) is None
    # the mixed-precision workload has its own figure (complex64 update, half the bytes)
    t32 = bench.measured_traffic("qep_n1024_16x16_mixed", "fp32", fpl)
    assert t32 is None or (t is not None and 0.3 * t < t32 < 0.6 * t)


def test_executed_fraction_of_the_3m_update():
    r = bench.roofline(_stats(280.0, 280.0), "fp64")
    assert r["executed_frac"] == pytest.approx(0.75 * r["frac"])
    r = bench.roofline(_stats(280.0, 280.0), "fp32")
    assert r["executed_frac"] == pytest.approx(r["frac"])

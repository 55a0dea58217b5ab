"""Host logic of bench.py: the roofline of the sum stage, the traffic per
launch, and the refusal of several GPUs (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_roofline_all_far_pairs_against_the_fp32_peak():
    st = {"pairs": 1e9, "pairs_near": 0}
    r = bench._sum_roofline(st, 0.1)            # 1e9 pairs in 0.1 ms
    flops = bench.FLOPS_PER_PAIR * 1e9
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(flops / 1e-4 / 1e12)
    assert r["peak"] == pytest.approx(bench.MFMA_FP32 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])


def test_roofline_mixed_pairs_take_the_time_weighted_peak():
    near = 2.5e8
    st = {"pairs": 1e9, "pairs_near": near}
    r = bench._sum_roofline(st, 0.2)
    t_peak = bench.FLOPS_PER_PAIR * ((1e9 - near) / bench.MFMA_FP32 + near / bench.MFMA_FP64)
    assert r["peak"] == pytest.approx(bench.FLOPS_PER_PAIR * 1e9 / t_peak / 1e12)
    assert bench.MFMA_FP64 / 1e12 < r["peak"] < bench.MFMA_FP32 / 1e12
    assert r["frac"] == pytest.approx(t_peak / 2e-4)


def test_roofline_without_time_or_work():
    assert bench._sum_roofline({"pairs": 0, "pairs_near": 0}, 1.0)["frac"] is None
    assert bench._sum_roofline({"pairs": 10, "pairs_near": 0}, 0.0)["achieved"] is None


def test_traffic_per_launch_scales_the_per_step_counters():
    per_step = bench._k_sum_traffic("fp32far")
    assert per_step == pytest.approx(bench.K_SUM_TRAFFIC["read_bytes"] + bench.K_SUM_TRAFFIC["written_bytes"])
    assert bench._k_sum_traffic("fp32far", 8.0) == pytest.approx(8 * per_step)
    assert bench._k_sum_traffic("fp64", 8.0) is None


def test_several_gpus_are_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr

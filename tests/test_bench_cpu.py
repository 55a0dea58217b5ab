"""Host logic of bench.py: the rooflines of the two kernel sums, the traffic
per launch, the window starts and the refusal of several GPUs (no GPU needed)."""
import os
import subprocess
import sys

import numpy as np
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


def test_traffic_per_launch_adds_the_kernels_of_the_stage(monkeypatch):
    monkeypatch.setattr(bench, "K_SUM_TRAFFIC", None)
    assert bench._k_sum_traffic() is None
    monkeypatch.setattr(bench, "K_SUM_TRAFFIC", {"far": {"read_bytes": 3e6, "written_bytes": 5e6},
                                                 "near": {"read_bytes": 1e6, "written_bytes": 2e6}})
    assert bench._k_sum_traffic() == pytest.approx(11e6)


def test_valu_roofline_of_the_pair_by_pair_sum():
    # all pairs FP32: 13 issue slots each over 256 CUs x 64 lanes x 2.4 GHz
    r = bench._valu_roofline({"pairs": 1e9, "pairs_near": 0}, 1.0)
    assert r["bound"] == "alu" and r["unit"] == "pairs/s"
    assert r["peak"] == pytest.approx(256 * 64 * 2.4e9 / 13)
    assert r["achieved"] == pytest.approx(1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    # a quarter of the pairs FP64 at 28 slots: the time-weighted peak lies between
    r = bench._valu_roofline({"pairs": 1e9, "pairs_near": 2.5e8}, 1.0)
    assert 256 * 64 * 2.4e9 / 28 < r["peak"] < 256 * 64 * 2.4e9 / 13
    assert bench._valu_roofline({"pairs": 0, "pairs_near": 0}, 1.0)["frac"] is None


def test_start_steps_leave_room_for_the_window():
    class Sc:
        n_steps = np.array([500, 4000, 120, 64])

    class Wl:
        scan = Sc()
    s = bench._start_steps(Wl(), 65, seed=1)
    assert (s >= 0).all() and (s + 65 <= np.maximum(Sc.n_steps, 65)).all()
    assert np.array_equal(s, bench._start_steps(Wl(), 65, seed=1))


def test_several_gpus_are_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_load_point_share_counts_the_faces_that_feed_the_step():
    from paper_2511_20432_amd import workloads as W
    # 64 x 32 x 16 elements, 3 x 3 points per face element: the top face
    # (64 x 32 elements) holds 2 of the 7 parts of the boundary points
    patch = W.block_patch((0, 0, 0), (4e-3, 2e-3, 1e-3), (64, 32, 16), 3)
    assert bench.load_point_share(patch) == pytest.approx(5.0 / 7.0, rel=1e-15)

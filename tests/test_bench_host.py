"""Host logic of bench.py, no GPU: the one-GPU contract, the roofline record
and the lookup of counter-measured HBM traffic keyed by kernel source."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _metrics(dominant):
    return {"dominant": dominant, "dominant_achieved_GBps": 4000.0, "bytes_per_launch": 5368709120,
            "dominant_tflops": 39.3, "dominant_flops_per_launch": 50465865728,
            "dominant_ms": 1.3}


def test_roofline_of_the_fused_pass_is_alu_bound_with_hbm_beside():
    r = bench.roofline(_metrics("sweep_xy"), 123)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == bench.PEAK_VALU_TFLOPS
    assert r["frac"] == pytest.approx(39.3 / 78.6, abs=1e-4)
    assert r["traffic"] == 123
    assert r["hbm"]["unit"] == "GB/s" and r["hbm"]["frac"] == pytest.approx(0.5)
    # achieved = algorithmic flops per launch / mean launch time
    assert 376 * 512 ** 3 == r["flops_per_launch_algorithmic"]


def test_roofline_of_a_single_sweep_is_hbm_bound():
    r = bench.roofline(_metrics("sweep_z"), None)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == bench.PEAK_HBM_GBS
    assert r["frac"] == pytest.approx(0.5) and r["traffic"] is None


def test_flops_per_cell_is_the_sum_of_the_counted_steps():
    # slopes and Hancock half step 88, HLLC face flux 74, update 15
    assert bench.FLOPS_PER_CELL_AXIS == 88 + 74 + 15


def test_traffic_is_reported_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    data = {"sweep_xy@w": {"bytes_per_launch": 11, "source_hash": h},
            "sweep_z@w": {"bytes_per_launch": 22, "source_hash": "0" * 16}}
    (tmp_path / "traffic.json").write_text(json.dumps(data))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.measured_traffic("sweep_xy", "w") == 11
    assert bench.measured_traffic("sweep_z", "w") is None      # other sources
    assert bench.measured_traffic("sweep_x", "w") is None      # never measured


def test_source_hash_covers_every_kernel_source():
    names = sorted(os.listdir(bench.CSRC))
    assert any(n.endswith(".hip") for n in names)
    assert len(bench.kernel_source_hash()) == 16

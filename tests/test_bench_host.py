"""Host-side logic of bench.py (CPU only): the one-GPU refusal, the traffic
figure read from the committed counter summaries (and dropped once the leaf
sources differ from the ones the counters were taken on), and the power
sampler's summary of its samples."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("mode", ["bf16x3", "f32", "fp8"])
def test_traffic_from_committed_profiles(mode):
    """The committed summaries were taken on the current leaf sources: their
    calibrated bytes per launch come back as the roofline's traffic."""
    t = bench.traffic_from_profiles(mode, "normal_f32_16384")
    assert t is not None and 1e8 < t < 1e11
    assert bench.traffic_from_profiles("f64", "normal_f32_16384") is None       # no summary for FP64
    assert bench.traffic_from_profiles(mode, "square_f32_8192") is None         # nor for this workload


def test_traffic_dropped_when_sources_change(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hpp"
    src.write_text("// a different kernel source\n")
    monkeypatch.setattr(bench, "LEAF_KERNEL_FILES", [str(src)])
    monkeypatch.setattr(bench, "ROOT", ROOT)
    assert bench.traffic_from_profiles("bf16x3", "normal_f32_16384") is None


def test_power_summary_keeps_the_samples_under_load():
    p = bench.PowerSampler(False)
    assert p.summary() is None
    # idle samples at the start and end of the region, and the loaded ones
    p.samples = [(250.0, 150.0), (1340.0, 1780.0), (1350.0, 1790.0), (1345.0, 1785.0), (260.0, 160.0)]
    s = p.summary()
    assert s["samples"] == 3
    assert s["socket_w_median"] == 1345.0 and s["gfx_mhz_median"] == 1785.0

"""bench.py's contract on the host: the refusal of several GPUs, the work accounting behind the
roofline figures, and the use of the committed HBM-traffic summary."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_work_per_point_bin_is_the_documented_count():
    # (FP64 flops, FP32 flops, transcendental ops) per (point, bin) at three detectors
    assert bench.work_per_point_bin(3, True) == (16 + 3 * 3, 3 * 8, 3 * 2)
    assert bench.work_per_point_bin(3, False) == (94, 0, 0)
    assert bench.work_per_point_bin(3, False, grad=True) == (16 + 3 * 18 + 14 * 3 - 1 + 16, 0, 0)
    f64, f32, tr = bench.work_per_point_bin(3, True, grad=True)
    assert (f64, f32, tr) == (25, 14 * 3 - 1 + 16, 6)


def test_roofline_fraction_is_one_at_the_model_minimum_time():
    nd, nbins, npts = 3, 16225, 65536
    f64, f32, tr = bench.work_per_point_bin(nd, True)
    tmin = nbins * npts * (f64 / bench.PEAK_FP64 + f32 / bench.PEAK_FP32 + tr / bench.PEAK_TRANS)
    achieved, peak, frac = bench.roofline(nd, True, nbins, npts, tmin)
    assert frac == pytest.approx(1.0, rel=1e-12)
    assert achieved == pytest.approx(peak, rel=1e-12)
    _, _, half = bench.roofline(nd, True, nbins, npts, 2 * tmin)
    assert half == pytest.approx(0.5, rel=1e-12)


def test_traffic_summary_is_used_only_for_its_kernel_source_and_layout(tmp_path, monkeypatch):
    layout = bench.layout_key({"waves": 16, "groups": 1, "setup": False})
    assert layout == "W16G1S0"
    f = tmp_path / "traffic.txt"
    f.write_text(f"launch_layout: {layout}\nhbm_bytes_per_launch: 1.25e+08\n"
                 f"kernel_source_sha256_16: {bench.kernel_hash()}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.read_traffic(layout) == pytest.approx(1.25e8)
    assert bench.read_traffic("W8G2S1") is None                  # another launch layout
    f.write_text(f"launch_layout: {layout}\nhbm_bytes_per_launch: 1.25e+08\nkernel_source_sha256_16: 0123\n")
    assert bench.read_traffic(layout) is None                    # counters taken on other kernel sources


def test_committed_traffic_summary_parses():
    import os
    if not os.path.exists(bench.TRAFFIC_FILE):
        pytest.skip("no HBM counter summary committed for the evaluation kernel")
    text = open(bench.TRAFFIC_FILE).read()
    layout = text.split("launch_layout:")[1].split()[0]
    if bench.kernel_hash() not in text:
        pytest.skip("the kernel sources changed since the traffic counters were taken")
    assert bench.read_traffic(layout) == pytest.approx(float(text.split("hbm_bytes_per_launch:")[1].split()[0]))

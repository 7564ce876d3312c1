"""Host logic of bench.py (no GPU): the one-GPU refusal, the per-point
figures of the roofline, and the gating of the counter-measured traffic on
the kernel sources it was taken on."""
import os
import re
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
    assert r.stdout == ""


def test_per_point_figures():
    # 55 flops per WENO face and direction (3 faces), 6 divergence, 13 psi'
    # Laplacian, 26 fourth differences, 7 RHS, 9 line recurrences
    assert bench.x_pass_flops_per_point() == 226
    # element accesses per substage 6, 7, 6, averaged, times the element size
    assert bench.x_pass_bytes_per_point(4) == pytest.approx(19 / 3 * 4)
    assert bench.step_bytes_per_point(8) == 34 * 8
    assert bench.VALU_PEAK_TFLOPS == pytest.approx(256 * 4 * 16 * 2 * 2.4e9 / 1e12, rel=1e-3)


def test_traffic_is_reported_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    text = open(bench.TRAFFIC_FILE).read()
    recorded = re.search(r"^source-hash:\s*(\w+)", text, re.M).group(1)
    nbytes = float(re.search(r"^traffic-bytes-per-launch:\s*(\S+)", text, re.M).group(1))
    assert nbytes > 0
    got = bench.measured_traffic()
    assert got == (nbytes if recorded == bench.x_source_hash() else None)
    # a summary taken on other sources is ignored
    other = tmp_path / "t.md"
    other.write_text(text.replace(recorded, "0" * 16))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(other))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None

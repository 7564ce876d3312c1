"""Host logic of bench.py (no GPU): the one-GPU refusal, the per-point
figures of the roofline, and the gating of the counter-measured traffic and
instruction counts on the kernel sources they were taken on."""
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


def test_issue_rate_from_the_counted_instructions(tmp_path):
    # one wave64 VALU instruction per SIMD every 4 cycles: 16 lanes per cycle
    assert bench.VALU_ISSUE_PEAK == pytest.approx(256 * 4 * 16 * 2.4e9)
    text = open(bench.SQ_FILE).read()
    recorded = re.search(r"^source-hash:\s*(\w+)", text, re.M).group(1)
    n = float(re.search(r"^x-pass-valu-lane-instructions-per-launch:\s*(\S+)", text,
                        re.M).group(1))
    # the count is the table's SQ_INSTS_VALU of the x pass times 64 lanes
    waves = float(re.search(r"^\| SQ_INSTS_VALU \| (\S+) \|", text, re.M).group(1))
    assert n == pytest.approx(64 * waves, rel=1e-3)
    v = bench.issue_view(100.0)
    if recorded != bench.x_source_hash():
        assert v is None
    else:
        assert v["valu_lane_instructions_per_launch"] == n
        assert v["frac"] == pytest.approx(n / 1e-4 / bench.VALU_ISSUE_PEAK, rel=1e-3)
    other = tmp_path / "s.md"
    other.write_text(text.replace(recorded, "0" * 16))
    assert bench.issue_view(100.0, str(other)) is None
    assert bench.issue_view(100.0, str(tmp_path / "missing.md")) is None


def test_limiter_compares_issue_with_hbm_at_copy_rate():
    issue = {"frac": 0.9}
    # 4.9e8 bytes in 100 us: 4.9 TB/s, the copy rate
    assert bench.limiter(issue, 4.9e8, 100.0)["limiter"] == "hbm"
    got = bench.limiter(issue, 4.0e8, 100.0)
    assert got["limiter"] == "valu_issue"
    assert got["hbm_frac_of_copy_rate"] == pytest.approx(4.0e8 / 1e-4 / 1e9 / bench.COPY_GBS,
                                                         rel=1e-3)
    assert bench.limiter(None, 4.0e8, 100.0) is None
    assert bench.limiter(issue, None, 100.0) is None


def test_roofline_and_step_fractions():
    # 16.78 M points at 25.33 B each in 100 us: 4.25 TB/s
    r = bench.x_roofline(100.0, 256 ** 3, 4, traffic=5e8)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(256 ** 3 * 19 / 3 * 4)
    assert r["achieved"] == pytest.approx(256 ** 3 * 19 / 3 * 4 / 1e-4 / 1e9, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert r["traffic"] == 5e8
    # 34 elements per point per step
    f = bench.step_hbm_frac(256 ** 3, 4, 0.5, extra_bytes=1e8)
    assert f == pytest.approx((136 * 256 ** 3 + 1e8) / 5e-4 / 8e12, rel=1e-3)


def test_fp32_error_summary_and_drop_pdf():
    import numpy as np
    rng = np.random.default_rng(0)
    C64 = rng.uniform(size=(8, 8, 8))
    C32 = C64 + 1e-6
    roots = np.array([0, 40, 90])
    d64 = (roots, np.array([100, 30, 8]))
    d32 = (roots[:2], np.array([101, 30]))
    e = bench.fp32_errors(C32, C64, (2.0, 2.0 + 1e-9), (2.0, 2.0), d32, d64, 0.5, 4.0, 7)
    assert e["steps"] == 7
    assert e["l2_rel"] == pytest.approx(1e-6 * np.sqrt(C64.size) / np.linalg.norm(C64), rel=1e-6)
    assert e["mass_drift_fp32"] == pytest.approx(5e-10) and e["mass_drift_fp64"] == 0.0
    assert e["drop_volume_err"] == pytest.approx(abs(131 - 138) / 138)
    assert e["drops"]["matched_by_root"] == 2
    assert e["drops"]["max_rel_volume_err_fp32_vs_fp64"] == pytest.approx(0.01)
    pdf = e["drops"]["D_over_H_pdf_fp64"]
    assert pdf["drops"] == 3 and sum(pdf["counts"]) == 3
    width = pdf["edges"][1] - pdf["edges"][0]
    assert sum(pdf["pdf"]) * width == pytest.approx(1.0, rel=1e-3)
    dmax = np.cbrt(6 * 100 * 0.125 / np.pi) / 4.0
    assert pdf["max"] == pytest.approx(dmax)

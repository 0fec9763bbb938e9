"""CPU checks of bench.py's bookkeeping: the HBM traffic it reports comes from
the committed rocprofv3 summary only while that summary was measured on the
current library sources (sha256 over csrc), and the JSON contract refuses more
than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_follows_the_source_digest(monkeypatch, tmp_path):
    d = tmp_path / "profiles"
    d.mkdir()
    (d / "unbounded256_curl_fp32_hbm_counters.md").write_text(
        "# x\n\n    source_sha256: %s\n    traffic_bytes: sandwich_x 100 23\n    traffic_bytes: inv_y 7 8\n"
        % bench.kernel_source_digest())
    monkeypatch.setattr(bench, "PROFILES", str(d))
    assert bench.measured_traffic("sandwich_x", 256) == 123.0
    assert bench.measured_traffic("inv_y", 256) == 15.0
    assert bench.measured_traffic("c2r_z", 256) is None
    assert bench.measured_traffic("sandwich_x", 128) is None  # no file for that size
    (d / "unbounded256_curl_fp32_hbm_counters.md").write_text(
        "    source_sha256: %s\n    traffic_bytes: sandwich_x 100 23\n" % ("0" * 64))
    assert bench.measured_traffic("sandwich_x", 256) is None  # other sources


def test_committed_profile_parses():
    path = os.path.join(ROOT, "profiles", "unbounded256_curl_fp32_hbm_counters.md")
    text = open(path).read()
    assert "source_sha256:" in text and "traffic_bytes: sandwich_x" in text
    text = open(os.path.join(ROOT, "profiles", "unbounded256_curl_fp32_kernel_trace.md")).read()
    assert "source_sha256:" in text and "kernel_avg_us: sandwich_x" in text


def test_committed_profiles_match_the_kernel_sources():
    # the committed counters describe the kernels built from these sources
    for name in ("unbounded256_curl_fp32_hbm_counters.md", "unbounded256_curl_fp32_kernel_trace.md"):
        digest, _ = bench._profile_lines(os.path.join(ROOT, "profiles", name))
        assert digest == bench.kernel_source_digest(), name


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_profiled_kernel_time_follows_the_source_digest(monkeypatch, tmp_path):
    d = tmp_path / "profiles"
    d.mkdir()
    (d / "unbounded256_curl_fp32_kernel_trace.md").write_text(
        "# x\n\n    source_sha256: %s\n    kernel_avg_us: sandwich_x 650.5\n" % bench.kernel_source_digest())
    monkeypatch.setattr(bench, "PROFILES", str(d))
    assert bench.profiled_kernel_us("sandwich_x", 256) == 650.5
    assert bench.profiled_kernel_us("inv_y", 256) is None
    v = bench._profile_view("sandwich_x", 256, 2.0e9)
    assert abs(v["achieved"] - 2.0e9 / 650.5e-6 / 1e9) < 1e-9
    assert abs(v["frac"] - v["achieved"] / bench.HBM_PEAK_GBS) < 1e-12
    (d / "unbounded256_curl_fp32_kernel_trace.md").write_text(
        "    source_sha256: %s\n    kernel_avg_us: sandwich_x 650.5\n" % ("0" * 64))
    assert bench.profiled_kernel_us("sandwich_x", 256) is None
    assert bench._profile_view("sandwich_x", 256, 2.0e9) is None


def test_six_field_model_bytes():
    # 256^3, FP32: P1 0.60 + P2 1.21 + P3 2.56 (nine spectral fields and the
    # FP64 octant of 257^3) + P4 2.43 + P5 1.19 GB
    b = bench.six_field_model_bytes(256)
    K = 257
    A = K * 256 * 256 * 8
    B = K * 512 * 256 * 8
    assert b == 3 * (256 ** 3 * 4 + A) + 3 * (A + B) + 9 * B + K ** 3 * 8 + 6 * (B + A) + 6 * (A + 256 ** 3 * 4)
    assert 8.01e9 < b < 8.02e9

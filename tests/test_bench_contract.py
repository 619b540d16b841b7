"""Host-side parts of the benchmark: it refuses more than one GPU before
touching a device, and it reports a stored per-launch HBM byte count only for
the kernel named and only while the kernel sources match the digest stored
with it."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _summary(tmp_path, digest):
    d = tmp_path / "profiles"
    d.mkdir()
    (d / "hbm_traffic_w.md").write_text(
        "# HBM traffic per launch: `w`\n\n"
        "| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | HBM bytes per launch (calibrated) |\n"
        "|---|---|---|---|---|\n"
        "| `gemm_f64_kernel<64, 128, 16, 2, 4>` | 8 | 10 | 2 | 2.2528e+04 |\n"
        "| `reduce_kernel` | 4 | 1 | 1 | 3.0720e+03 |\n\n"
        f"sources_sha256: {digest}\n")


def test_traffic_read_for_matching_digest_and_kernel(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_digest", lambda: "abc")
    _summary(tmp_path, "abc")
    # kernel names match with or without the spaces rocprofv3 prints
    assert bench.profiled_traffic("gemm_f64_kernel<64,128,16,2,4>", "w") == 22528.0
    assert bench.profiled_traffic("reduce_kernel", "w") == 3072.0
    assert bench.profiled_traffic("gemm_f64_kernel<32,32,16,1,1>", "w") is None
    assert bench.profiled_traffic("gemm_f64_kernel<64,128,16,2,4>", "other") is None


def test_traffic_withheld_when_sources_changed(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_digest", lambda: "changed")
    _summary(tmp_path, "abc")
    assert bench.profiled_traffic("gemm_f64_kernel<64,128,16,2,4>", "w") is None


"""Host-side checks of bench.py (no GPU needed)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("// header\n__global__ void k(float* x) {\n    x[0] = 1.0f;  // set\n}\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    h0 = bench.kernel_source_sha256()
    src.write_text("// a different header\n__global__ void k(float* x) {\n"
                   "    x[0] = 1.0f;   // reworded comment\n}\n")
    assert bench.kernel_source_sha256() == h0
    src.write_text("// header\n__global__ void k(float* x) {\n    x[0] = 2.0f;  // set\n}\n")
    assert bench.kernel_source_sha256() != h0


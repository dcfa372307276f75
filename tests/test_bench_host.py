"""Host logic of bench.py (CPU): the HBM traffic figure of the dominant
kernel comes from the committed rocprofv3 summary only while the kernel
sources it lists are the ones the counters were taken on, and the benchmark
refuses more than one GPU."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_committed_summary_matches_the_sources():
    traffic = bench.profile_traffic("fp32_gemm_8192_sweep.md")
    assert traffic is not None, "kernel sources changed since the summary's counters were taken"
    # well above the 0.81 GB the 8192^3 product must move, well below 8 TB/s x 8 ms
    assert 0.8e9 < traffic < 64e9


def _summary(root, sources, digest):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    with open(os.path.join(root, "profiles", "k.md"), "w") as f:
        f.write("# summary\n\ntraffic_bytes_per_launch: 1234.0\n")
        f.write(f"sources: {' '.join(sources)}\nsource_hash: {digest}\n")


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("kernel text\n")
    digest = hashlib.sha256(b"kernel text\n").hexdigest()[:16]
    _summary(str(tmp_path), ["kernel.hip"], digest)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profile_traffic("k.md") == 1234.0
    src.write_text("kernel text, changed\n")   # a changed kernel: no figure
    assert bench.profile_traffic("k.md") is None
    assert bench.profile_traffic("missing.md") is None


def test_one_gpu_only():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)

"""Host logic of bench.py (no GPU): the traffic figure is taken from the
committed counter summary only while that summary matches the kernel sources
and the nodes per thread of the timed launch; multi-GPU runs are refused."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _summary(path, sha, npl, nbytes):
    with open(path, "w") as f:
        f.write("# header line: with a colon that must be ignored\n")
        f.write(f"hbm_bytes_per_launch: {nbytes}\nkernel_source_sha256_16: {sha}\nfield_npl: {hex(npl)}\n")


def test_traffic_figure_requires_matching_sources_and_field_layout(tmp_path, monkeypatch):
    path = str(tmp_path / "traffic.txt")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", path)
    assert bench.traffic_per_launch(0x42) is None  # no summary
    _summary(path, bench.kernel_hash(), 0x42, 137000000)
    assert bench.traffic_per_launch(0x42) == 137000000.0
    assert bench.traffic_per_launch(0x22) is None  # another field layout
    _summary(path, "0" * 16, 0x42, 137000000)
    assert bench.traffic_per_launch(0x42) is None  # taken on other sources


def test_kernel_hash_is_stable_and_short():
    h = bench.kernel_hash()
    assert h == bench.kernel_hash() and len(h) == 16 and int(h, 16) >= 0


def test_multi_gpu_run_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)

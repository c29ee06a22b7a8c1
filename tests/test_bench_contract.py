"""The benchmark's host-side contract, on the CPU: it refuses more than one
GPU with a message, its algorithmic-byte model is the one the roofline
uses, and the stored traffic figure is only used while it belongs to the
current kernel source."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_of_one_iteration():
    import bench
    # 32 B per vertex (y read, v read+write, y write) and 8 B per edge
    assert bench.alg_bytes(1_400_000, 2, 1) == 78_400_000
    assert bench.alg_bytes(70_000, 5, 1) == 32 * 70_000 + 8 * 70_000 * 6


def test_stored_traffic_belongs_to_the_current_kernel(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "step.hip"
    src.write_text("// kernel source\n")
    prof = tmp_path / "traffic.md"
    monkeypatch.setattr(bench, "STEP_SOURCES", [str(src)])
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(prof))
    prof.write_text(f"source_sha1: {bench.source_digest([str(src)])}\nhbm_bytes_per_launch: 4.5e+08\n")
    assert bench.stored_traffic() == pytest.approx(4.5e8)
    src.write_text("// kernel source, edited\n")
    assert bench.stored_traffic() is None
    os.remove(prof)
    assert bench.stored_traffic() is None


def test_committed_traffic_profile_matches_the_step_kernel():
    import bench
    assert bench.stored_traffic() is not None, "profiles/step_det_C3_traffic.md is stale for the det kernel"

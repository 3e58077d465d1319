"""Host-side logic of bench.py (no GPU): the stored counter traffic is used
only for the kernel variant and sources it was measured on, and the
multi-GPU request is refused."""
import json
import subprocess
import sys

import pytest

import bench


@pytest.fixture()
def traffic_file(tmp_path, monkeypatch):
    path = tmp_path / "solve_traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    return path


def _entry(kernel, hash_=None):
    return {"kernel": kernel, "kernel_hash": hash_ or bench.kernel_hash(), "hbm_bytes_per_launch": 1.5e13}


def test_traffic_matches_variant_and_layout(traffic_file):
    traffic_file.write_text(json.dumps({
        "water64/mixed": _entry("void k_solve_mixed<3, 4, 1024, 2, false, false, true>"),
        "water64/fp64": _entry("void k_solve<3, 3, 1024, 1, false, false, false>"),
    }))
    assert bench.stored_traffic("water64", "mixed", 1024, 2, 2) == 1.5e13
    assert bench.stored_traffic("water64", "fp64", 1024, 1, 1) == 1.5e13
    # another load depth, workgroup size or layout than the one measured
    assert bench.stored_traffic("water64", "mixed", 1024, 1, 2) is None
    assert bench.stored_traffic("water64", "fp64", 512, 1, 1) is None
    assert bench.stored_traffic("water64", "mixed", 1024, 2, 1) is None
    assert bench.stored_traffic("water64", "fp64", 1024, 1, 2) is None
    # layout 3 (both layouts, per sphere class): no single kernel was measured
    assert bench.stored_traffic("water64", "mixed", 1024, 2, 3) is None
    assert bench.stored_traffic("water128", "mixed", 1024, 2, 2) is None


def test_traffic_is_dropped_when_the_kernel_sources_change(traffic_file):
    traffic_file.write_text(json.dumps({
        "water64/mixed": _entry("void k_solve_mixed<3, 4, 1024, 2, false, false, true>", hash_="0" * 16)}))
    assert bench.stored_traffic("water64", "mixed", 1024, 2, 2) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "GPU" in (r.stdout + r.stderr)

"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the
algorithmic byte count behind roofline.achieved, and the lookup of the
counter-measured HBM traffic, which is reported only for the native
sources and launch shape it was measured with."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_unit():
    """One sample of length d = 3 (two interior vertices): 16 B per expanded
    vertex, 8 B per scanned entry, 8 B per predecessor edge, 20 B per newly
    visited vertex, 8 (d + 1) B of backtrack reads, 4 (d - 1) B of counter
    updates."""
    r = {"samples": 1, "vertices_expanded": 5, "edges_scanned": 100, "pred_edges": 3, "vertices_visited": 7,
         "path_vertices": 2}
    assert bench.algorithmic_bytes(r) == 16 * 5 + 8 * 100 + 8 * 3 + 20 * 7 + 8 * 4 + 4 * 2
    # linear in the work: two copies of the same work cost twice the bytes
    r2 = {k: 2 * v for k, v in r.items()}
    assert bench.algorithmic_bytes(r2) == 2 * bench.algorithmic_bytes(r)


@pytest.fixture
def fake_profile(tmp_path, monkeypatch):
    os.makedirs(tmp_path / "profiles")
    prof = {"kernel": "k_sample<1024, true>", "csrc_sha256": "abc", "block_size": 1024, "epoch_size": 2304,
            "traffic_bytes_per_dispatch": 5.5e9}
    (tmp_path / "profiles" / "k_sample_w_traffic.json").write_text(json.dumps(prof))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return monkeypatch


def test_traffic_reported_for_the_profiled_sources_and_shape(fake_profile):
    fake_profile.setattr(bench, "csrc_sha256", lambda: "abc")
    assert bench.counter_traffic("w", 2304, 1024) == 5.5e9
    assert bench.counter_traffic("w", 4608, 1024) is None     # another epoch size
    assert bench.counter_traffic("w", 2304, 512) is None      # another workgroup size
    assert bench.counter_traffic("other", 2304, 1024) is None  # no profile for that workload


def test_traffic_withheld_once_the_sources_change(fake_profile):
    fake_profile.setattr(bench, "csrc_sha256", lambda: "def")
    assert bench.counter_traffic("w", 2304, 1024) is None

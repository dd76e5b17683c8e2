"""Host-side logic of the benchmark (no GPU): the multi-GPU refusal and the
lookup of recorded HBM traffic, which must drop the figure as soon as the
kernel's sources change."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU only" in p.stdout + p.stderr


def _write_record(root, src_text, sha=None):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    os.makedirs(os.path.join(root, "k"), exist_ok=True)
    with open(os.path.join(root, "k", "kernel.hip"), "w") as f:
        f.write(src_text)
    rec = {"kernel": "k_levels", "workload": "wc-100m", "sources": ["k/kernel.hip"],
           "sources_sha256": sha or hashlib.sha256(src_text.encode()).hexdigest(),
           "traffic_bytes_per_launch": 12345}
    with open(os.path.join(root, "profiles", "x_hbm_traffic.md"), "w") as f:
        f.write("# t\n\ntraffic-record: " + json.dumps(rec) + "\n")


def test_traffic_record_matches_sources(tmp_path, monkeypatch):
    _write_record(str(tmp_path), "kernel v1")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_levels", "wc-100m") == 12345
    assert bench.measured_traffic("k_levels", "seq-20m") is None    # another workload
    assert bench.measured_traffic("k_flow", "wc-100m") is None      # no record for that kernel
    assert bench.measured_traffic(None, "wc-100m") is None


def test_traffic_record_dropped_after_a_source_change(tmp_path, monkeypatch):
    _write_record(str(tmp_path), "kernel v1")
    with open(os.path.join(str(tmp_path), "k", "kernel.hip"), "a") as f:
        f.write("// changed\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_levels", "wc-100m") is None


"""Host-side checks of bench.py that need no GPU: the multi-GPU request is refused
with a message, and the committed HBM-counter record belongs to the current
forward kernel source (otherwise the benchmark reports traffic as null)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_follows_kernel_sources(tmp_path, monkeypatch):
    """A kernel's counter record counts only while the kernel's sources are the ones
    it was taken with: bench.py reports the bytes then, and null (None) after any
    change to them."""
    rec = {"kernels": {k: {"source_hash": bench.source_hash(k), "bytes_per_launch": 1.0e9 + i}
                       for i, k in enumerate(bench.KERNEL_SOURCES)}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    for i, k in enumerate(bench.KERNEL_SOURCES):
        assert bench.measured_traffic(k) == 1.0e9 + i
    rec["kernels"]["adj_kernel"]["source_hash"] = "0" * 16
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic("adj_kernel") is None
    assert bench.measured_traffic("fwd_kernel") == 1.0e9


def test_committed_profiles_name_their_commands():
    """Every committed rocprofv3 summary gives the command that made it, which runs
    committed files only (bench.py)."""
    prof = os.path.join(ROOT, "profiles")
    names = [n for n in os.listdir(prof) if n.endswith(".md")]
    assert names
    for name in names:
        txt = open(os.path.join(prof, name)).read()
        assert "rocprofv3" in txt and "bench.py" in txt, name
        assert "_work" not in txt, name

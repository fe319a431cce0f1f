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


def test_traffic_record_matches_forward_source():
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    assert rec["source_hash"] == bench.fwd_source_hash()
    assert rec["bytes_per_launch"] > 0
    assert bench.measured_traffic() == rec["bytes_per_launch"]
    # the counter and trace summaries name the commands that produced them
    for name in ("fwd_kernel_c3_kernel_trace.md", "fwd_kernel_c3_hbm_traffic.md"):
        txt = open(os.path.join(ROOT, "profiles", name)).read()
        assert "rocprofv3" in txt and "bench.py" in txt

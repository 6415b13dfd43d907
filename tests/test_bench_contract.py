"""The benchmark's command-line contract, on the CPU: one GPU only (any
--gpus above 1 exits with status 2 and a message, before touching a device),
and the helpers that label its roofline line."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_recorded_traffic_matches_kernel_source():
    # the committed counter summary is used only for the gridding source it
    # was taken on (its stored hash must equal the current one to be read)
    sys.path.insert(0, ROOT)
    import bench
    txt = open(bench.PMC_FILE).read()
    stored = [ln.split(":", 1)[1].strip() for ln in txt.splitlines() if ln.startswith("kernel_source_sha:")]
    assert stored, "counter summary lacks its source hash"
    if stored[0] == bench.grid_kernel_hash():
        assert bench.recorded_traffic() > 0
    else:
        assert bench.recorded_traffic() is None

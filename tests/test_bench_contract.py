"""bench.py's host-side contract (no device work): more than one GPU is refused
with a message, and the traffic note parses only for the current stencil source."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_stored_traffic_matches_the_stencil_source():
    sys.path.insert(0, ROOT)
    import bench
    note = os.path.join(ROOT, "profiles", "wave_step_hbm_traffic.md")
    if not os.path.exists(note):
        pytest.skip("no traffic note")
    v = bench.stored_traffic("wave_step_blocked", "c256", "float32")
    # either the counters were taken with this source (a positive byte count), or the source
    # changed since and bench reports null
    assert v is None or v > 2.6e8
    assert bench.stored_traffic("wave_step_blocked", "c999", "float32") is None

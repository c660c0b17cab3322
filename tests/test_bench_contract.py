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
    """Every counter line of the traffic note is returned for its kernel, workload and
    precision exactly while the stencil source is the one it was taken with (else
    None), and lies between the launch's compulsory bytes (5 words per voxel: p(k),
    p(k-1) and k' read, two planes of results written) and 1.5 times that."""
    import hashlib
    import re
    sys.path.insert(0, ROOT)
    import bench
    note = os.path.join(ROOT, "profiles", "wave_step_hbm_traffic.md")
    if not os.path.exists(note):
        pytest.skip("no traffic note")
    src = os.path.join(ROOT, "paper_1901_06503_amd", "csrc", "kernels_wave.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    rows = re.findall(r"^traffic: kernel=(\S+) recipe=(\S+) dtype=(\S+) bytes_per_launch=([0-9.eE+]+) "
                      r"source_sha256=([0-9a-f]+)", open(note).read(), flags=re.M)
    assert rows, "the note holds no counter lines"
    edges = {"c128": 128, "c256": 256, "c384": 384}
    for kernel, recipe, dtype, value, taken_with in rows:
        got = bench.stored_traffic(kernel, recipe, dtype)
        assert got == (float(value) if taken_with == sha else None), (kernel, recipe, dtype)
        compulsory = 5 * (8 if dtype == "float64" else 4) * edges[recipe] ** 3
        assert compulsory <= float(value) <= 1.5 * compulsory, (kernel, recipe, dtype, float(value) / compulsory)
    assert bench.stored_traffic(rows[0][0], "c999", rows[0][2]) is None
    assert bench.stored_traffic("no_such_kernel", rows[0][1], rows[0][2]) is None

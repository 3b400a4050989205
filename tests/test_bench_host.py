"""Host-side checks of bench.py (no GPU): the one-GPU guard, the algorithmic
bytes of the roofline, and the machine-read traffic records of the
committed counter summary."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_phase_bytes_are_one_record_read_and_written():
    w = {"d": 3, "n": 1 << 24}
    pb = bench.phase_bytes(w)
    assert pb["sort"] == pb["split"] == pb["scatter"] == 32 * (1 << 24)


def test_traffic_records_parse_and_match_a_data_pass():
    with open(bench.TRAFFIC_SUMMARY) as f:
        recs = [re.match(r"traffic-record: kernel=(\S+) bytes_per_launch=(\d+) source_sha256=([0-9a-f]{64})$", l.strip())
                for l in f if l.startswith("traffic-record:")]
    assert recs and all(recs)
    kinds = {m.group(1) for m in recs}
    assert {"scatter", "split", "sort"} <= kinds
    # every data pass moves at least its algorithmic 32 B per particle at N = 2^24
    assert all(int(m.group(2)) >= 32 * (1 << 24) for m in recs)
    # the bench reports a record only for the sources it was measured on
    t = bench.measured_traffic("sort")
    assert t is None or t == int([m for m in recs if m.group(1) == "sort"][0].group(2))

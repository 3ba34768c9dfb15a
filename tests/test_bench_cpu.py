"""Host-side contract of bench.py (no GPU): one GPU only, and the HBM-traffic record of the dominant
kernel is reported only while its sources are the ones the counters were taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


DEFAULT_LAUNCH = {"fwd_mode": 0, "bwd_chunk_mul": 1}


def test_traffic_record_matches_the_committed_sources():
    got = bench.traffic_bytes(256, DEFAULT_LAUNCH)
    assert got is not None and got > 0
    # the algorithmic traffic of one launch is ~157 MB; the record must be of that order
    assert 1.0e8 < got < 3.0e8
    # the forward's launch shape does not enter the adjoint kernel's traffic
    assert bench.traffic_bytes(256, dict(DEFAULT_LAUNCH, fwd_mode=1)) == got


def test_traffic_record_is_dropped_when_the_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "sources_digest", lambda: "0" * 64)
    assert bench.traffic_bytes(256, DEFAULT_LAUNCH) is None


def test_traffic_record_is_dropped_for_another_launch():
    """Another batch or chunk multiplier writes another number of partial rows."""
    assert bench.traffic_bytes(16, DEFAULT_LAUNCH) is None
    assert bench.traffic_bytes(256, dict(DEFAULT_LAUNCH, bwd_chunk_mul=2)) is None

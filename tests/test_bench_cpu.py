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


def _record():
    import json
    with open(bench.TRAFFIC_RECORD) as fh:
        for line in fh:
            if line.startswith("traffic-record: "):
                return json.loads(line[len("traffic-record: "):])
    return None


def test_traffic_record_is_reported_for_its_own_sources(monkeypatch):
    rec = _record()
    assert rec is not None
    # the committed sources: reported only if they are the ones the counters were taken on
    got = bench.traffic_bytes(rec["batch"], rec["launch"])
    assert (got is not None) == (rec["sources_sha256"] == bench.sources_digest())
    monkeypatch.setattr(bench, "sources_digest", lambda: rec["sources_sha256"])
    got = bench.traffic_bytes(rec["batch"], rec["launch"])
    # the algorithmic traffic of one launch is ~157 MB; the record must be of that order
    assert got is not None and 1.0e8 < got < 3.0e8
    # the forward's launch shape does not enter the adjoint kernel's traffic
    assert bench.traffic_bytes(rec["batch"], dict(rec["launch"], fwd_mode=1 - rec["launch"]["fwd_mode"])) == got


def test_traffic_record_is_dropped_when_the_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "sources_digest", lambda: "0" * 64)
    rec = _record()
    assert bench.traffic_bytes(rec["batch"], rec["launch"]) is None


def test_traffic_record_is_dropped_for_another_launch(monkeypatch):
    """Another batch, chunk multiplier or packing writes another number of partial rows."""
    rec = _record()
    monkeypatch.setattr(bench, "sources_digest", lambda: rec["sources_sha256"])
    assert bench.traffic_bytes(rec["batch"] // 16, rec["launch"]) is None
    other = 2 if rec["launch"]["bwd_chunk_mul"] != 2 else 4
    assert bench.traffic_bytes(rec["batch"], dict(rec["launch"], bwd_chunk_mul=other)) is None
    pack = rec["launch"].get("bwd_pack", 0)
    assert bench.traffic_bytes(rec["batch"], dict(rec["launch"], bwd_pack=1 - pack)) is None
    assert bench.traffic_bytes(rec["batch"], dict(rec["launch"], bwd_pack=pack)) is not None


def test_forward_traffic_record(monkeypatch):
    """The forward windows kernel's record: reported for its own sources, batch and launch mode."""
    rec = bench._read_record(bench.FWD_TRAFFIC_RECORD)
    assert rec is not None and rec["kernel"] == "k_windows_cl"
    monkeypatch.setattr(bench, "fwd_sources_digest", lambda: rec["sources_sha256"])
    got = bench.fwd_traffic_bytes(rec["batch"], rec["launch"])
    # coefficient rows, U rows, k scales and C of 256 points: tens of MB per launch
    assert got is not None and 2.0e7 < got < 2.0e8
    assert bench.fwd_traffic_bytes(rec["batch"] // 2, rec["launch"]) is None
    assert bench.fwd_traffic_bytes(rec["batch"], {"fwd_mode": 1 - rec["launch"]["fwd_mode"]}) is None
    monkeypatch.setattr(bench, "fwd_sources_digest", lambda: "0" * 64)
    assert bench.fwd_traffic_bytes(rec["batch"], rec["launch"]) is None


def test_contraction_flops():
    alg, issued = bench.contraction_flops(15, 103, 256, 1024)
    assert alg == 15 * 16 * 1024 * 103 * 256 and issued == 2 * 256 * 1024 * 103 * 256

"""Host-side logic of bench.py (no GPU): the recorded HBM traffic of the
dominant kernel is reported only while the kernel source is the one the
rocprofv3 counters were taken on."""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _summary(tmp_path, sha, traffic="123450000"):
    p = tmp_path / "traffic.md"
    p.write_text(f"# summary\n\ntraffic_bytes_per_launch: {traffic}\n\ndfgt.hip sha256 at measurement: {sha}\n")
    return str(p)


def test_traffic_reported_for_the_measured_source(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source A")
    sha = hashlib.sha256(b"kernel source A").hexdigest()
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _summary(tmp_path, sha))
    value, note = bench.recorded_traffic()
    assert value == 123450000.0
    assert "FETCH_SIZE" in note


def test_traffic_withheld_once_the_source_changes(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source B")
    sha = hashlib.sha256(b"kernel source A").hexdigest()
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _summary(tmp_path, sha))
    value, note = bench.recorded_traffic()
    assert value is None
    assert "changed" in note


def test_traffic_withheld_without_a_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    value, _ = bench.recorded_traffic()
    assert value is None


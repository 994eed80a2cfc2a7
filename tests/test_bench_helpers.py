"""Host logic of the benchmark's roofline: the measured HBM traffic per launch
is read from a committed counter summary only while the kernel sources still
hash to what the summary recorded, and the summary tool hashes sources the
same way."""
import hashlib
import os

import bench
import prof_window


def test_traffic_read_while_sources_unchanged(tmp_path, monkeypatch):
    root = str(tmp_path)
    (tmp_path / "k.hip").write_text("kernel source v1\n")
    sha = prof_window.sources_sha256(["k.hip"], root)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k_case.md").write_text(
        f"# summary\n\nTRAFFIC kernel=k bytes_per_launch=12345 sources=k.hip sha256={sha}\n")
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.measured_traffic("k") == 12345.0
    assert bench.measured_traffic("other") is None
    # a changed source voids the figure
    (tmp_path / "k.hip").write_text("kernel source v2\n")
    assert bench.measured_traffic("k") is None
    # a missing source too
    os.remove(tmp_path / "k.hip")
    assert bench.measured_traffic("k") is None


def test_summary_tool_and_benchmark_hash_alike(tmp_path):
    """Both hash the concatenated bytes of the listed sources in order."""
    (tmp_path / "a.hip").write_bytes(b"first\n")
    (tmp_path / "b.hpp").write_bytes(b"second\n")
    h = hashlib.sha256(b"first\nsecond\n").hexdigest()
    assert prof_window.sources_sha256(["a.hip", "b.hpp"], str(tmp_path)) == h

"""bench.py's readers of the committed counter summaries: figures are taken
only from a summary recorded on the current kernel sources."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write(path, sha, rows):
    with open(path, "w") as f:
        f.write("# header\n")
        f.write(f"kernel_sources_sha256_16: {sha}\n")
        f.write("workload | kernel | dispatches | fetch KiB | write KiB | r | w | traffic / algorithmic\n")
        for r in rows:
            f.write(r + "\n")


def test_large_traffic_read_from_a_summary_of_the_current_sources(tmp_path, monkeypatch):
    p = tmp_path / "large.txt"
    _write(p, bench.kernel_sources_hash(), [
        "carpet r9 compact (edge records) | k | 10 | 1 | 2 | 1.1 | 1.0 | 1.049",
        "carpet r9 box (19,683^2) | k | 7 | 1 | 2 | 1.1 | 1.0 | 1.077",
        "H r10 compact (byte scatter) | k | 10 | 1 | 2 | 1.1 | 1.0 | 1.053"])
    monkeypatch.setattr(bench, "LARGE_COUNTERS", str(p))
    assert bench.measured_large_traffic("carpet_r9") == (1.049, 1.077)
    assert bench.measured_large_traffic("hfractal_r10") == (1.053, None)
    assert bench.measured_large_traffic("triangle_r16") == (None, None)


def test_large_traffic_ignored_for_other_sources(tmp_path, monkeypatch):
    p = tmp_path / "large.txt"
    _write(p, "0123456789abcdef", ["carpet r9 compact | k | 10 | 1 | 2 | 1.1 | 1.0 | 1.049"])
    monkeypatch.setattr(bench, "LARGE_COUNTERS", str(p))
    assert bench.measured_large_traffic("carpet_r9") == (None, None)
    monkeypatch.setattr(bench, "LARGE_COUNTERS", str(tmp_path / "missing.txt"))
    assert bench.measured_large_traffic("carpet_r9") == (None, None)


def test_triangle_traffic_needs_the_current_sources(tmp_path, monkeypatch):
    p = tmp_path / "tri.txt"
    p.write_text(f"kernel_sources_sha256_16: {bench.kernel_sources_hash()}\nhbm_bytes_per_launch: 86952297\n")
    monkeypatch.setattr(bench, "COUNTERS", str(p))
    assert bench.measured_traffic(86093442) == 86952297.0
    p.write_text("kernel_sources_sha256_16: 0123456789abcdef\nhbm_bytes_per_launch: 86952297\n")
    assert bench.measured_traffic(86093442) is None

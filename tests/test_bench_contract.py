"""Host-side parts of the measurement script: the one-GPU guard and the reading of committed
counter summaries (no GPU needed)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_summaries_are_read_only_for_the_sources_they_were_measured_on(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    assert len(h) == 64
    good = tmp_path / "traffic.txt"
    good.write_text("hbm_traffic_over_algorithmic: 1.059\nkernel_source_sha256: %s\n" % h)
    stale = tmp_path / "stale.txt"
    stale.write_text("hbm_traffic_over_algorithmic: 1.059\nkernel_source_sha256: %s\n" % ("0" * 64))
    valu = tmp_path / "valu.txt"
    valu.write_text("valu_active_frac: 0.700\nkernel_source_sha256: %s\n" % h)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.committed_traffic_ratio() == 1.059
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.committed_traffic_ratio() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.committed_traffic_ratio() is None
    monkeypatch.setattr(bench, "VALU_FILE", str(valu))
    assert bench.committed_valu() == 0.7


def test_committed_summaries_match_the_current_sources():
    """The committed counter summaries (tile kernel, whole step) carry the hash of the kernel
    sources they were measured on; the bench reports their figures only while it matches."""
    assert bench.committed_traffic_ratio() is not None
    assert bench.committed_valu() is not None
    assert bench.committed_step_bytes() is not None

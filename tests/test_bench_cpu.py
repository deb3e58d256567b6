"""bench.py's host-side contract (no device): more than one GPU is refused
with a message, the HBM-traffic figure is read only while the executor
sources match the stored hash, and the stored exact values cover every seed
the throughput run uses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single-GPU" in r.stderr


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    assert bench.persist_traffic() is not None   # summary matches the sources
    stale = tmp_path / "summary.md"
    stale.write_text("kernel-sources-sha256: `%s`\nhbm-bytes-per-launch: `123`\n" % ("0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(stale))
    assert bench.persist_traffic() is None       # another kernel: no figure
    good = tmp_path / "good.md"
    good.write_text("kernel-sources-sha256: `%s`\nhbm-bytes-per-launch: `123`\n"
                    % bench.persist_sources_sha256())
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(good))
    assert bench.persist_traffic() == 123


def test_stored_values_cover_every_seed():
    want = bench.golden_sg16()
    assert set(range(bench.N_SEEDS)) <= set(want)

"""bench.py's host-side contract (no device): more than one GPU is refused
with a message, the HBM-traffic figure is read only while the executor
sources match the stored hash, the stored values cover every seed the runs
use, and the configuration checks agree with the oracle's."""
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
    stale = tmp_path / "summary.md"
    stale.write_text("kernel-sources-sha256: `%s`\nhbm-bytes-per-launch: `123`\n" % ("0" * 64))
    for kernel in ("persist", "tgemm"):
        srcs = bench.TRAFFIC[kernel][1]
        monkeypatch.setitem(bench.TRAFFIC, kernel, (str(stale), srcs))
        assert bench.kernel_traffic(kernel) is None       # another kernel: no figure
        good = tmp_path / ("good_%s.md" % kernel)
        good.write_text("kernel-sources-sha256: `%s`\nhbm-bytes-per-launch: `123`\n"
                        % bench.sources_sha256(kernel))
        monkeypatch.setitem(bench.TRAFFIC, kernel, (str(good), srcs))
        assert bench.kernel_traffic(kernel) == 123
    assert bench.kernel_traffic("gather") is None


def test_stored_values_cover_every_seed():
    want = bench.golden_sg16()
    assert set(range(bench.N_SEEDS)) <= set(want)
    # the headline's seeds 0-19 and the King's subgraph leg's seeds
    assert set(range(20)) <= set(bench.golden_values("sg32_values.txt"))
    assert set(range(8)) <= set(bench.golden_values("ksg40_values.txt"))


def test_configuration_checks():
    import instances as I
    from oracle import config
    g = I.spin_glass_square(6, 3)
    rng = __import__("numpy").random.default_rng(1)
    for _ in range(5):
        s = rng.choice([-1, 1], size=g["n"])
        assert bench.energy_sg(s, g["edges"], g["J"]) == config.spin_glass_energy(
            s, g["edges"], g["J"], None)
    k = I.kings_subgraph(6, 2)
    x = __import__("numpy").zeros(k["n"], dtype=int)
    assert bench.independent_weight(x, k["edges"]) == 0
    u, v = k["edges"][0]
    x[u] = x[v] = 1
    assert bench.independent_weight(x, k["edges"]) is None

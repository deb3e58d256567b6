"""Small-step forests on the host (no device): the forest planned for a step
program, and in place for the keep-all program of configuration recovery,
is run with the executor's addressing rules and compared buffer by buffer
with a plain contraction of the same steps; every offset is bounds-checked
(tests/forest_check.cpp, g++; the product's host sources, the HIP runtime
library linked but no device call made)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_05470_amd", "csrc")
SOURCES = ["tree.cpp", "search.cpp", "plan.cpp", "network.cpp", "crt.cpp", "persist.cpp",
           "prof.cpp"]


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    gxx = shutil.which("g++")
    lib = "/opt/rocm/lib"
    if gxx is None or not os.path.isdir("/opt/rocm/include") or not os.path.isdir(lib):
        pytest.skip("g++ or ROCm is missing")
    out = str(tmp_path_factory.mktemp("forest") / "forest_check")
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-D__HIP_PLATFORM_AMD__",
           "-I", CSRC, "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
           os.path.join(ROOT, "tests", "forest_check.cpp")]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    cmd += ["-o", out, "-L", lib, "-Wl,-rpath," + lib, "-lamdhip64", "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def _run(exe, tmp_path, kind, n, edges, w, lt, refine, vw=None):
    edges = np.asarray(edges).reshape(-1, 2)
    lines = ["%d %d %d %d %d 0" % (kind, n, len(edges), lt, refine)]
    lines += ["%d %d %d" % (a, b, x) for (a, b), x in zip(edges, w)]
    if kind == 1:
        lines.append(" ".join(str(int(x)) for x in vw))
    p = tmp_path / "inst.txt"
    p.write_text("\n".join(lines) + "\n")
    r = subprocess.run([exe, str(p)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]
    assert r.stdout.startswith("ok"), r.stdout


@pytest.mark.parametrize("L,t,refine", [(12, 8, 0), (14, 9, 4), (10, 0, 0)])
def test_spin_glass_forests(exe, tmp_path, L, t, refine):
    """Branching (leaf groups with shared subtrees and deferred slicing) and
    one whole contraction (t = 0: every step runs once, in the forest when
    small)."""
    g = I.spin_glass_square(L, 1)
    _run(exe, tmp_path, 0, g["n"], g["edges"], g["J"], t if t > 0 else 30, refine)


def test_kings_subgraph_forests(exe, tmp_path):
    g = I.kings_subgraph(10, 2, weights="1..10")
    e = np.asarray(g["edges"]).reshape(-1, 2)
    _run(exe, tmp_path, 1, g["n"], e, np.zeros(len(e), np.int64), 7, 4, vw=g["w"])

"""The host planner (network build, greedy and refined orders, branch-and-
bound search, step programs with and without deferred slicing and keep-all)
built with AddressSanitizer and UndefinedBehaviorSanitizer from the library's
host sources and run on several topologies: any out-of-bounds access, use
after free or undefined arithmetic fails the test.  Host code only, g++."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_05470_amd", "csrc")
SOURCES = ["tree.cpp", "search.cpp", "plan.cpp", "network.cpp", "crt.cpp"]


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are missing")
    out = str(tmp_path_factory.mktemp("asan") / "host_planner_check")
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__",
           "-I", CSRC, "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
           os.path.join(ROOT, "tests", "host_planner_check.cpp")]
    cmd += [os.path.join(CSRC, s) for s in SOURCES] + ["-o", out, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def _run(exe, tmp_path, kind, n, edges, w, lt, refine, vonly=0, vw=None):
    edges = np.asarray(edges).reshape(-1, 2)
    lines = ["%d %d %d %d %d %d" % (kind, n, len(edges), lt, refine, vonly)]
    lines += ["%d %d %d" % (a, b, x) for (a, b), x in zip(edges, w)]
    if kind == 1:
        lines.append(" ".join(str(int(x)) for x in vw))
    p = tmp_path / "inst.txt"
    p.write_text("\n".join(lines) + "\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe, str(p)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.startswith("ok"), r.stdout


@pytest.mark.parametrize("refine", [0, 4])
def test_square_lattice(exe, tmp_path, refine):
    g = I.spin_glass_square(12, 3)
    _run(exe, tmp_path, 0, g["n"], g["edges"], g["J"], 8, refine)


def test_refined_root_joining_fixed_subtrees(exe, tmp_path):
    """16x16 at T_target = 2^10 with refined orders: the case whose root
    joins a subtree of fixed variables only (it once made the planner write
    before its buffer table)."""
    g = I.spin_glass_square(16, 0)
    _run(exe, tmp_path, 0, g["n"], g["edges"], g["J"], 10, 8)


def test_values_only_and_rectangle(exe, tmp_path):
    g = I.spin_glass_rect(8, 11, 2)
    _run(exe, tmp_path, 0, g["n"], g["edges"], g["J"], 7, 4, vonly=1)


def test_kings_subgraph_weighted(exe, tmp_path):
    g = I.kings_subgraph(9, 1, weights="1..10")
    _run(exe, tmp_path, 1, g["n"], g["edges"], np.zeros(len(np.asarray(g["edges"]).reshape(-1, 2)),
         np.int64), 6, 4, vw=g["w"])


def test_random_regular_and_cubic(exe, tmp_path):
    g = I.spin_glass_random_regular(40, 5)
    _run(exe, tmp_path, 0, g["n"], g["edges"], g["J"], 6, 4)
    g = I.spin_glass_cubic(3, 3, 4, 2)
    _run(exe, tmp_path, 0, g["n"], g["edges"], g["J"], 6, 4)

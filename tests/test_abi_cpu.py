"""The C-ABI library loads and exports every symbol include/bbtn.h declares
(no compute calls: CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bbtn.h")
LIB = os.path.join(ROOT, "paper_2602_05470_amd", "libbbtn.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bbtn_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for must in ("bbtn_create", "bbtn_destroy", "bbtn_solve_spinglass", "bbtn_solve_mwis",
                 "bbtn_tgemm", "bbtn_gather", "bbtn_reduce", "bbtn_bound"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_all_declared_symbols():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_declares_same_names():
    import paper_2602_05470_amd as B
    assert sorted(B.EXPORTS) == sorted(n for n in declared() if n in B.EXPORTS)
    assert set(declared()) <= set(B.EXPORTS) | {"bbtn_result", "bbtn_options"}


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_default_options_and_struct_sizes():
    import paper_2602_05470_amd as B
    lib = B.load()
    o = B._Options()
    lib.bbtn_default_options(ctypes.byref(o))
    assert o.residues_per_pass == 3 and o.branching == 1 and o.batched == 1


def test_options_and_result_layout_match_the_header(tmp_path):
    """The binding's ctypes structures have the C layout of include/bbtn.h
    (sizes and the offsets of every field), checked with the host C compiler."""
    import shutil
    import subprocess
    import paper_2602_05470_amd as B
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "bbtn.h"', "int main(void) {"]
    for ct, name in ((B._Options, "bbtn_options"), (B._Result, "bbtn_result")):
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for f in ct._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f[0], name, f[0]))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                   text=True).stdout.splitlines())
    for ct, name in ((B._Options, "bbtn_options"), (B._Result, "bbtn_result")):
        assert int(got[name]) == ctypes.sizeof(ct), name
        for f in ct._fields_:
            assert int(got[name + "." + f[0]]) == getattr(ct, f[0]).offset, (name, f[0])

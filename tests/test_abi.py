"""The C-ABI library loads on the host and exports every entry point that
include/sw.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2505_18743_amd", "libswdg.so")
HDR = os.path.join(ROOT, "include", "sw.h")


def declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(?:sw_status|void|const char\s*\*)\s*(sw_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("sw_create", "sw_apply_operator", "sw_rk_stage", "sw_step", "sw_set_bathymetry"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_the_same_symbols():
    from paper_2505_18743_amd.binding import EXPORTS, load
    load()
    assert sorted(EXPORTS) == declared()


def test_struct_layouts_match_the_header(tmp_path):
    """Field offsets of the ctypes mirrors equal those gcc computes from sw.h."""
    import shutil
    import subprocess
    from paper_2505_18743_amd.binding import SwAmrParams, SwAmrStats, SwDiag, SwMeshDesc, SwParams
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"sw_mesh_desc": SwMeshDesc, "sw_params": SwParams, "sw_diag": SwDiag,
               "sw_amr_params": SwAmrParams, "sw_amr_stats": SwAmrStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sw.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln.strip():
            a, b, v = ln.split()
            got[(a, b)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)

"""The C-ABI library builds for gfx950, loads, and exports every function the
header declares (no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^(?:int|void|const char\*)\s+(gv_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["gv_init", "gv_configure", "gv_transport", "gv_stats", "gv_ledger", "gv_trace", "gv_n_cells",
              "gv_finalize", "gv_last_error", "gv_debug_step"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2005_00949_amd as gv
    if not os.path.exists(gv.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(gv.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n


def test_calls_before_init_fail_cleanly():
    import paper_2005_00949_amd as gv
    if not os.path.exists(gv.LIB_PATH):
        pytest.skip("library not built")
    lib = gv.load()
    lib.gv_finalize()
    st = gv.Stats()
    assert lib.gv_stats(ctypes.byref(st)) == 5       # GV_E_NOT_INIT
    assert b"gv_init" in lib.gv_last_error()
    assert lib.gv_transport(None, 0, 0, None) == 5


def test_missing_library_raises(monkeypatch, tmp_path):
    import paper_2005_00949_amd as gv
    monkeypatch.setattr(gv, "_lib", None)
    monkeypatch.setattr(gv, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        gv.load()


def test_binding_struct_layouts_match_header(tmp_path):
    """Every ctypes mirror has the size and field offsets the C compiler gives
    the header's struct (compiled here with gcc against include/gv.h)."""
    import shutil
    import subprocess

    import paper_2005_00949_amd as gv
    if not shutil.which("gcc"):
        pytest.skip("no C compiler")
    mirrors = {"gv_material": gv.Material, "gv_geometry": gv.Geometry, "gv_tables": gv.Tables,
               "gv_config": gv.Config, "gv_stats_t": gv.Stats, "gv_trace_rec": None, "gv_debug_io": gv.DebugIO}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gv.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        if py is not None:
            for fname, _ in py._fields_:
                lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for cname, py in mirrors.items():
        if py is None:
            assert got[(cname, "size")] == gv.TRACE_DTYPE.itemsize
            continue
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)

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

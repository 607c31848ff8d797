"""The C-ABI library loads and exports every function include/sharp.h declares
(no GPU needed: only the shared object is opened)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sharp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("sim_create", "sim_set_state", "sim_advance", "sim_get_state", "sim_destroy"):
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_1905_03917_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1905_03917_amd import build
        build.build()
    lib = ctypes.CDLL(P.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTS) == _declared()


def test_binding_refuses_to_run_without_library(tmp_path, monkeypatch):
    import paper_1905_03917_amd as P
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(P, "_lib", None)
    with pytest.raises(RuntimeError):
        P.lib()


def test_binding_constants_match_the_header():
    """the integer #defines of the header and the binding's copies agree"""
    import paper_1905_03917_amd as P
    txt = open(os.path.join(ROOT, "include", "sharp.h")).read()
    defs = dict(re.findall(r"#define\s+(SIM_[A-Z_]+)\s+(-?\d+)\b", txt))
    assert "SIM_GRAPH_MAX_CELLS" in defs
    for name, val in defs.items():
        if hasattr(P, name):
            assert getattr(P, name) == int(val), name

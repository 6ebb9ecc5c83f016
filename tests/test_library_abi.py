"""CPU checks of the C-ABI library: it loads and exports every function that
include/giem.h declares (no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "giem.h")
LIB = os.path.join(ROOT, "paper_1512_06126_amd", "lib", "libgiem.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*(giem_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for n in ("giem_tables", "giem_apply", "giem_solve", "giem_adjoint", "giem_fields",
              "giem_tables_import", "giem_tables_export", "giem_free", "giem_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_symbol_list_matches_header():
    import paper_1512_06126_amd as g
    assert sorted(g.exported_symbols()) == declared_functions()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1512_06126_amd as g
    monkeypatch.setattr(g, "LIBPATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(g, "_lib", None)
    with pytest.raises(ImportError):
        g.load()

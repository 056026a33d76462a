"""The C-ABI library builds and exports every function include/mmdeig.h declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mmdeig.h")
LIB = os.path.join(ROOT, "paper_1804_03415_amd", "libmmdeig.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("mmd_build", "eig_leftmost", "mmd_free", "mmd_last_error", "mmd_apply",
              "mmd_solve", "mmd_info", "mmd_export", "mmdk_spmm"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_all_symbols():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_error_path_without_device_work():
    import paper_1804_03415_amd as m
    L = m.lib()
    L.mmd_free(None)  # NULL is ignored
    rc = L.mmd_info(None, None, None, None, None, None)
    assert rc == 1 and b"null handle" in L.mmd_last_error()

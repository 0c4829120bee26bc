"""The C-ABI library loads and exports every entry point the header
declares (no GPU work: nothing is called but the string functions)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vrsplat.h")
LIB = os.path.join(ROOT, "paper_2410_17932_amd", "libvrsplat.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vrs_[a-z0-9_]+)\s*\(", src)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"missing exports: {missing}"
    lib.vrs_version.restype = ctypes.c_char_p
    lib.vrs_status_string.restype = ctypes.c_char_p
    assert b"gfx950" in lib.vrs_version()
    assert lib.vrs_status_string(2) == b"workspace capacity exceeded"


def test_python_binding_names_match_header():
    from paper_2410_17932_amd import api
    assert set(api.SIGNATURES) == set(declared())

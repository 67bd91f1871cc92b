"""The C-ABI library loads and exports every symbol include/edx.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "edx.h")
LIB = os.path.join(ROOT, "paper_2105_06806_amd", "libedx.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(edx_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("edx_build_sector", "edx_hv", "edx_lanczos_ground_state", "edx_green_cf"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libedx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libedx.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.edx_status_str.restype = ctypes.c_char_p
    assert lib.edx_status_str(0) == b"EDX_OK"
    assert lib.edx_status_str(4) == b"EDX_E_NOCONV"
    assert lib.edx_status_str(99) == b"EDX_E_UNKNOWN"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libedx.so not built")
def test_binding_names_match_header():
    # the Python binding declares a signature for every header function it wraps
    import importlib.util
    spec = importlib.util.spec_from_file_location("edx_sigs", os.path.join(ROOT, "paper_2105_06806_amd", "edx.py"))
    txt = open(spec.origin).read()
    for n in ("edx_build_sector", "edx_hv", "edx_lanczos_ground_state", "edx_green_cf"):
        assert f'"{n}"' in txt

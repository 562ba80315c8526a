"""The C-ABI library loads and exports every entry point include/gazemap.h declares
(no compute: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gazemap.h")
LIB = os.path.join(ROOT, "paper_2601_07571_amd", "libgazemap.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


def test_header_declares_the_three_named_calls():
    names = declared_functions()
    for n in ("build_surface_samples", "accumulate_density", "gm_scene_create", "gm_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), f"missing export {n}"
    import paper_2601_07571_amd as gm
    assert set(gm.SYMBOLS) <= set(declared_functions())
    lib.gm_version.restype = ctypes.c_int32
    assert lib.gm_version() >> 16 == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_errors_without_gpu():
    """Argument checks run before any device call."""
    lib = ctypes.CDLL(LIB)
    lib.gm_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    st = lib.gm_scene_create(None, 0, ctypes.byref(h))
    assert st == -1 and b"n_meshes" in lib.gm_last_error()
    st = lib.accumulate_density(None, None, None, None, ctypes.c_int64(0), None, ctypes.c_double(1.0),
                                ctypes.c_uint32(0), None, None, None, None)
    assert st == -1

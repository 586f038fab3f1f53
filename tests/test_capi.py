"""The C-ABI library loads and exports every entry point its header declares (no GPU needed;
no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vbx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(vbx_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1611_03631_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    return b.LIB


def test_header_declares_entry_points():
    names = declared_functions()
    for core in ("vbx_map_create", "vbx_integrate", "vbx_export_blocks", "vbx_integrate_batch",
                 "vbx_integrate_multi"):
        assert core in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_lists_every_declared_symbol():
    import paper_1611_03631_amd as vbx
    assert sorted(vbx.EXPORTED) == declared_functions()


def test_status_strings_without_gpu(libpath):
    lib = ctypes.CDLL(libpath)
    lib.vbx_status_string.restype = ctypes.c_char_p
    assert lib.vbx_status_string(-3) == b"block pool full"
    assert lib.vbx_status_string(0) == b"ok"


def test_library_has_no_oracle_code(libpath):
    """The product library never contains the oracle's symbols."""
    out = open(libpath, "rb").read()
    assert b"orc_integrate" not in out and b"orc_dda" not in out


def test_interpolate_rejects_bad_arguments_before_any_device_work(libpath):
    """A NULL map, or NULL buffers with points to query, are refused on the host."""
    lib = ctypes.CDLL(libpath)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.vbx_map_interpolate.argtypes = [vp, vp, sz, vp]
    lib.vbx_map_interpolate.restype = ctypes.c_int
    import paper_1611_03631_amd as vbx
    assert lib.vbx_map_interpolate(None, None, 0, None) == vbx.ERR_INVALID_ARG
    assert lib.vbx_map_interpolate(None, None, 5, None) == vbx.ERR_INVALID_ARG

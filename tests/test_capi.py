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


def test_binding_declares_argument_types_of_every_entry_point(libpath):
    """ctypes passes undeclared integer arguments as 32-bit ints: a pointer argument would be
    truncated.  Every declared function that takes arguments has its argument types set."""
    import paper_1611_03631_amd as vbx
    L = vbx.lib()
    src = open(os.path.join(ROOT, "include", "vbx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    missing = []
    for name in declared_functions():
        m = re.search(name + r"\s*\(([^)]*)\)", src)
        takes_args = m is not None and m.group(1).strip() not in ("", "void")
        if takes_args and getattr(L, name).argtypes is None:
            missing.append(name)
    assert not missing, f"no argtypes: {missing}"


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


def _create_ex(libpath):
    lib = ctypes.CDLL(libpath)
    lib.vbx_map_create_ex.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.vbx_map_create_ex.restype = ctypes.c_int
    lib.vbx_default_params.argtypes = [ctypes.c_void_p]
    lib.vbx_default_params.restype = None
    return lib


def test_allocator_hook_returning_null_fails_create_cleanly(libpath):
    """A map whose allocator hook returns NULL is not created: VBX_ERR_OUT_OF_MEMORY, the out
    parameter untouched, and nothing handed to the free hook (the hook's allocation is the map's
    first device request, so no device is needed to see this)."""
    import paper_1611_03631_amd as vbx
    lib = _create_ex(libpath)
    asked, freed = [], []
    alloc = vbx.ALLOC_FN(lambda n, ctx: asked.append((n, ctx)) or None)
    free = vbx.FREE_FN(lambda ptr, ctx: freed.append(ptr))
    p = vbx.MapParams()
    lib.vbx_default_params(ctypes.byref(p))
    p.alloc, p.free, p.alloc_ctx = alloc, free, 77
    out = ctypes.c_void_p(1234)
    assert lib.vbx_map_create_ex(ctypes.byref(p), ctypes.byref(out)) == vbx.ERR_OUT_OF_MEMORY
    assert out.value == 1234
    assert len(asked) == 1 and asked[0][1] == 77 and asked[0][0] > 0
    assert freed == []


def test_allocator_hook_needs_both_functions(libpath):
    import paper_1611_03631_amd as vbx
    lib = _create_ex(libpath)
    p = vbx.MapParams()
    lib.vbx_default_params(ctypes.byref(p))
    alloc = vbx.ALLOC_FN(lambda n, ctx: None)
    p.alloc = alloc
    out = ctypes.c_void_p(None)
    assert lib.vbx_map_create_ex(ctypes.byref(p), ctypes.byref(out)) == vbx.ERR_INVALID_ARG
    assert out.value is None


def test_storage_modes_are_validated(libpath):
    """The 16-bit storages hold W as binary16: a W_max above 65504 is refused, as is an unknown
    storage code."""
    import paper_1611_03631_amd as vbx
    lib = _create_ex(libpath)
    for storage, w_max in ((vbx.F16, 7e4), (vbx.S16, 7e4), (3, 1e4)):
        p = vbx.MapParams()
        lib.vbx_default_params(ctypes.byref(p))
        p.storage, p.w_max = storage, w_max
        out = ctypes.c_void_p(None)
        assert lib.vbx_map_create_ex(ctypes.byref(p), ctypes.byref(out)) == vbx.ERR_INVALID_ARG

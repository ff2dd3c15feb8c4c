"""The C-ABI library loads on the CPU and exports every entry point include/gm.h declares
(no compute calls: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for core in ("gm_bin", "gm_render_stacks", "gm_render_volume", "gm_backward", "gm_adam_step"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2603_00145_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libgm.so not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared()) == set(_lib.EXPORTED)


def test_host_only_calls():
    from paper_2603_00145_amd import _lib
    lib = _lib.load()
    assert lib.gm_abi_version() == 4
    assert _lib.tile_dims() == (16, 16, 4)
    # host-side validation needs no device
    g = _lib.GmGrid()
    g.nx, g.ny, g.nz = 0, 4, 4
    st = lib.gm_bin_query(10, ctypes.byref(g), 1, 0, None, None, None)
    assert st == _lib.GM_ERR_INVALID_ARGUMENT
    assert b"dims" in lib.gm_last_error()
    g.nx = 4
    for i in range(3):
        g.world_to_index[4 * i + i] = 2.0
    tt = ctypes.c_int64()
    sb = ctypes.c_size_t()
    assert lib.gm_bin_query(10, ctypes.byref(g), 1, 100, None, ctypes.byref(tt), ctypes.byref(sb)) == 0
    assert tt.value == 1 and sb.value > 0
    assert lib.gm_adam_step(None, None, None, None, 4, 1e-3, 0.9, 0.999, 1e-8, 0, None) == \
        _lib.GM_ERR_INVALID_ARGUMENT

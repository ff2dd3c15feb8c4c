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
    assert lib.gm_abi_version() == 5
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


def test_host_validation_of_the_extension_entry_points():
    """Host-side checks of the SSIM, pose, lattice and binning entry points (they return
    before anything is launched, so no device is needed)."""
    from paper_2603_00145_amd import _lib
    lib = _lib.load()
    P = ctypes.c_void_p
    fake = P(0x1000)           # never dereferenced on the host
    arr = (P * 2)(fake, fake)
    dims = (ctypes.c_int32 * 6)(8, 8, 2, 8, 8, 2)
    # SSIM: stack count, lambda, negative dims
    assert lib.gm_loss_ssim(0, arr, arr, dims, 0.5, arr, fake, fake, None) == _lib.GM_ERR_INVALID_ARGUMENT
    assert lib.gm_loss_ssim(2, arr, arr, dims, float("nan"), arr, fake, fake, None) == \
        _lib.GM_ERR_INVALID_ARGUMENT
    bad = (ctypes.c_int32 * 6)(8, -1, 2, 8, 8, 2)
    assert lib.gm_loss_ssim(2, arr, arr, bad, 0.5, arr, fake, fake, None) == _lib.GM_ERR_INVALID_ARGUMENT
    assert b"dims" in lib.gm_last_error()
    # lattice refinement: sizes and the old lattice's count
    g = _lib.GmGaussians(27, fake, fake, fake, fake)
    assert lib.gm_upsample_lattice(0, ctypes.byref(g), 4, fake, fake, fake, fake, None) == \
        _lib.GM_ERR_INVALID_ARGUMENT
    assert lib.gm_upsample_lattice(4, ctypes.byref(g), 4, fake, fake, fake, fake, None) == \
        _lib.GM_ERR_INVALID_ARGUMENT
    assert b"g_old^3" in lib.gm_last_error()
    # pose gradient: NULL Gaussians
    assert lib.gm_grid_pose_grads(None, None, None, 0, fake, fake, 0, None) == \
        _lib.GM_ERR_INVALID_ARGUMENT
    # block query: a cell resolution of 0 is refused before any launch
    grid = _lib.GmGrid()
    grid.nx, grid.ny, grid.nz = 16, 16, 4
    c, s_ = 0.8, 0.6
    grid.world_to_index[0], grid.world_to_index[1] = 8 * c, -8 * s_
    grid.world_to_index[4], grid.world_to_index[5] = 8 * s_, 8 * c
    grid.world_to_index[10] = 2.0
    b = _lib.GmBins()
    b.n_grids, b.n_gauss, b.capacity_pairs = 1, 27, 1000
    for f in ("records", "tile_count", "box_volume", "tile_start", "pair_gauss", "scratch"):
        setattr(b, f, 0x1000)
    b.scratch_bytes = 1 << 30
    npairs = ctypes.c_int64()
    opts = _lib.GmBinOpts(3.0, 2, 0)
    st = lib.gm_bin(ctypes.byref(g), ctypes.byref(grid), 1, ctypes.byref(opts), ctypes.byref(b),
                    ctypes.byref(npairs), None)
    assert st == _lib.GM_ERR_INVALID_ARGUMENT


def test_host_validation_of_the_multi_grid_field_backward():
    """The multi-grid field backward sizes its workspace for every grid's points rounded up
    to 16, refuses grid counts outside [1, GM_MAX_GRIDS] and returns before any launch when
    no grid has a point."""
    from paper_2603_00145_amd import _lib
    lib = _lib.load()
    P = ctypes.c_void_p
    fake = 0x1000
    nrf = _lib.GmNrf(16, 3, 64, 128, 0.1, 0, fake, fake, fake, fake, fake, fake)
    npts = (ctypes.c_int64 * 3)(3001, 17, 0)
    got, one = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.gm_nrf_workspace_grids(ctypes.byref(nrf), 3, npts, ctypes.byref(got)) == 0
    assert lib.gm_nrf_workspace(ctypes.byref(nrf), 3008 + 32, ctypes.byref(one)) == 0
    assert got.value == one.value
    assert lib.gm_nrf_workspace_grids(ctypes.byref(nrf), 0, npts, ctypes.byref(got)) == \
        _lib.GM_ERR_INVALID_ARGUMENT
    assert lib.gm_nrf_workspace_grids(ctypes.byref(nrf), _lib.GM_MAX_GRIDS + 1, npts,
                                      ctypes.byref(got)) == _lib.GM_ERR_INVALID_ARGUMENT
    grids = (_lib.GmGrid * 2)()
    for g in grids:
        g.nx, g.ny, g.nz = 8, 8, 2
        for i in range(3):
            g.world_to_index[4 * i + i] = 1.0
    idx = (P * 2)(P(fake), P(fake))
    dl = (P * 2)(P(fake), P(fake))
    sc = (ctypes.c_float * 2)(1.0, 1.0)
    zero = (ctypes.c_int64 * 2)(0, 0)
    gr = _lib.GmNrfGrads(fake, fake, fake, fake, fake, fake)
    assert lib.gm_nrf_backward_grids(ctypes.byref(nrf), 2, grids, idx, zero, dl, sc,
                                     ctypes.byref(gr), None, 0, None) == 0
    # no points and no index list (an empty sample): nothing to do
    none = (P * 2)(P(0), P(0))
    assert lib.gm_nrf_backward_grids(ctypes.byref(nrf), 2, grids, none, zero, dl, sc,
                                     ctypes.byref(gr), None, 0, None) == 0
    # a grid with no idx must name every voxel; errors name the grid
    idx[1] = P(0)
    bad = (ctypes.c_int64 * 2)(5, 7)
    assert lib.gm_nrf_backward_grids(ctypes.byref(nrf), 2, grids, idx, bad, dl, sc,
                                     ctypes.byref(gr), None, 0, None) == \
        _lib.GM_ERR_INVALID_ARGUMENT
    assert b"grid 1" in lib.gm_last_error()
    sc[0] = float("inf")
    assert lib.gm_nrf_backward_grids(ctypes.byref(nrf), 1, grids, idx, bad, dl, sc,
                                     ctypes.byref(gr), None, 0, None) == \
        _lib.GM_ERR_INVALID_ARGUMENT
    assert b"scale" in lib.gm_last_error()


def test_index_to_world_follows_the_stated_recipe():
    """gm_index_to_world (a host call) gives, bit for bit, the adjugate recipe its header
    states, which the oracle writes out on its own (the residual field's coordinates depend on
    the last bit of this matrix)."""
    import numpy as np
    from oracle import nrf as onrf
    from paper_2603_00145_amd import _lib, inputs
    rng = np.random.default_rng(4)
    grids = [inputs.volume_grid(64)] + inputs.orthogonal_stacks(96, 24, 1.0, rng, 2.0, 1.0) + \
        inputs.oblique_stacks(80, 20, 1.25)
    for g in grids:
        got = _lib.index_to_world(g)
        ref = onrf.index_to_world(g.world_to_index)
        assert np.array_equal(got, ref), g.name

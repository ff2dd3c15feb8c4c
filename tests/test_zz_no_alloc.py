"""gm_render_loss_smooth_l1_noalloc (the loss partials in the library's static per-device array)
against gm_render_loss_smooth_l1 (the same partials in a caller workspace), both through the
C ABI: dL/dI, the stored renderings and the loss bit-identical, on two calls in a row, the
second on fewer tiles than the first, so that stale partials of the first call would show."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2603_00145_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    from paper_2603_00145_amd import _lib, api
    api.load()
    return _lib, api


def problem(seed, n, n_g, nz):
    rng = np.random.default_rng(seed)
    g = inputs.init_anisotropic(n, n_g, rng)
    grids = [inputs.stack_grid("axial", n, nz[0], 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("coronal", n, nz[1], 1.0),
             inputs.stack_grid("sagittal", n, nz[2], 1.0)]
    targ = [rng.normal(0.3, 1.0, size=gr.shape).astype(np.float32) for gr in grids]
    return g, grids, targ


def noalloc(lib_mod, api, b, ids, targets, outs, dl):
    loss = torch.full((4,), float("nan"), dtype=torch.float32, device="cuda")
    idarr = (ctypes.c_int32 * len(ids))(*ids)
    st = lib_mod.load().gm_render_loss_smooth_l1_noalloc(
        ctypes.byref(b.struct()), idarr, len(ids),
        api.ptr_array([t.data_ptr() for t in targets]),
        api.ptr_array([t.data_ptr() for t in outs]),
        api.ptr_array([d.data_ptr() for d in dl]),
        ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    api.check(st)
    return loss[0]


@pytest.mark.parametrize("big,small", [((61, 2500, (17, 13, 15)), (23, 300, (6, 5, 7)))])
def test_noalloc_equals_workspace_entry(mods, big, small):
    lib_mod, api = mods
    for call, (n, n_g, nz) in enumerate((big, small)):
        g, grids, targ = problem(10 + call, n, n_g, nz)
        ids = [0, 1, 2]
        say(f"no-alloc call {call}: n={n} gaussians={n_g} nz={nz}")
        b = api.Bins(g.n, grids)
        b.bin(api.GaussParams.from_host(g))
        t = [torch.from_numpy(x).cuda() for x in targ]
        outs_ref = [torch.full(gr.shape, float("nan"), device="cuda") for gr in grids]
        loss_ref, dl_ref = api.render_loss(b, ids, t, outs=outs_ref)
        outs = [torch.full(gr.shape, float("nan"), device="cuda") for gr in grids]
        dl = [torch.full(gr.shape, float("nan"), device="cuda") for gr in grids]
        loss = noalloc(lib_mod, api, b, ids, t, outs, dl)
        torch.cuda.synchronize()
        for k in ids:
            assert torch.equal(outs[k], outs_ref[k]), f"call {call} grid {k}: rendering differs"
            assert torch.equal(dl[k], dl_ref[k]), f"call {call} grid {k}: dL/dI differs"
        lv, lr = float(loss), float(loss_ref)
        say(f"  loss no-alloc {lv!r} workspace {lr!r}")
        assert np.float32(lv).tobytes() == np.float32(lr).tobytes()


def test_noalloc_rejects_too_many_tiles(mods):
    """More tiles than the static array holds: an error before anything is enqueued."""
    lib_mod, api = mods
    n = 16 * 64
    grids = [inputs.volume_grid(n)]           # 64 x 64 x 256 = 1,048,576 tiles of 16x16x4
    g = inputs.init_anisotropic(n, 1, np.random.default_rng(0))
    b = api.Bins(g.n, grids, capacity=1024)
    b.bin(api.GaussParams.from_host(g))
    st = lib_mod.load().gm_render_loss_smooth_l1_noalloc(
        ctypes.byref(b.struct()), (ctypes.c_int32 * 1)(0), 1,
        api.ptr_array([0]), None, api.ptr_array([0]), None, None)
    assert st == lib_mod.GM_ERR_CAPACITY
    assert b"static scratch" in lib_mod.load().gm_last_error()

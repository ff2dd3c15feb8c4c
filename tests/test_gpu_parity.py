"""HIP path against the FP64 oracle, element by element, through the C ABI.

Bars: tile boxes, tile counts, pair totals and per-tile lists bit-exact; FP32 voxel values and
gradients within 1e-5 normwise relative (max |gpu - oracle| / max |oracle|, per output).
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import gauss, recipe
from paper_2603_00145_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    from paper_2603_00145_amd import api as _api
    _api.load()
    return _api


def normwise(gpu, ref):
    ref = np.asarray(ref, np.float64)
    d = np.max(np.abs(np.asarray(gpu, np.float64) - ref)) if ref.size else 0.0
    s = np.max(np.abs(ref)) if ref.size else 0.0
    return d / s if s > 0 else d


def ragged_problem(seed=0, n_g=700, n=37):
    rng = np.random.default_rng(seed)
    g = inputs.init_anisotropic(n, n_g, rng)
    grids = [inputs.stack_grid("axial", n, 11, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("coronal", n, 9, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("sagittal", n, 10, 1.0),
             inputs.volume_grid(n)]
    return g, grids, rng


def oracle_bins(g, grids, tile):
    """Boxes, counts, totals and CSR tile lists from the oracle's recipe."""
    out = []
    tiles_all, gids_all = [], []
    base = 0
    for gr in grids:
        lo, hi, ne, _ = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, gr)
        t, gi = recipe.tile_lists(lo, hi, ne, gr, tile, base)
        tiles_all.append(t)
        gids_all.append(gi)
        out.append((lo, hi, ne, recipe.tile_counts(lo, hi, ne, tile),
                    int(recipe.box_volume(lo, hi, ne).sum())))
        base += recipe.n_tiles(gr, tile)
    t = np.concatenate(tiles_all)
    gi = np.concatenate(gids_all)
    start, gids = recipe.csr_from_pairs(t, gi, base)
    return out, start, gids


def check_bins_exact(api, b, g, grids):
    from paper_2603_00145_amd import _lib
    tile = _lib.tile_dims()
    per, start, gids = oracle_bins(g, grids, tile)
    for k, (lo, hi, ne, cnt, vol) in enumerate(per):
        glo, ghi = (t.cpu().numpy() for t in b.boxes(k))
        gne = (glo <= ghi).all(1)
        assert np.array_equal(gne, ne), f"grid {k}: nonempty flags differ"
        assert np.array_equal(glo[ne], lo[ne]), f"grid {k}: lo differs"
        assert np.array_equal(ghi[ne], hi[ne]), f"grid {k}: hi differs"
        assert np.array_equal(b.tile_count[k, :g.n].cpu().numpy(), cnt), f"grid {k}: counts"
        assert b.pair_count(k) == vol, f"grid {k}: box volume"
    assert b.n_pairs == len(gids)
    assert np.array_equal(b.tile_start.cpu().numpy(), start)
    # each grid's list range as gm_bin reports it on the host
    per_grid = [int(cnt.sum()) for (_, _, _, cnt, _) in per]
    assert [int(b._s.list_start[k]) for k in range(len(grids) + 1)] == list(np.cumsum([0] + per_grid))
    raw = b.pair_gauss[:b.n_pairs].cpu().numpy().view(np.uint32)
    assert np.array_equal((raw & 0x7FFFFFFF).astype(np.int64), gids)
    # bit 31 marks exactly the entry whose tile holds the Gaussian's box lower corner
    T = np.asarray(tile)
    bases = np.cumsum([0] + [recipe.n_tiles(gr, tile) for gr in grids])
    entry_tile = np.repeat(np.arange(bases[-1]), np.diff(start))
    entry_grid = np.searchsorted(bases, entry_tile, side="right") - 1
    home = np.zeros((len(grids), g.n), np.int64)
    for k, ((lo, hi, ne, cnt, vol), gr) in enumerate(zip(per, grids)):
        ntx, nty = -(-gr.nx // T[0]), -(-gr.ny // T[1])
        t = lo // T
        home[k] = np.where(ne, bases[k] + (t[:, 2] * nty + t[:, 1]) * ntx + t[:, 0], -1)
    assert np.array_equal(raw >> 31 == 1, home[entry_grid, gids] == entry_tile)


@pytest.mark.parametrize("seed", [0, 1])
def test_bins_bit_exact_ragged(api, seed):
    g, grids, _ = ragged_problem(seed)
    say("bins ragged seed", seed)
    b = api.Bins(g.n, grids)
    b.bin(api.GaussParams.from_host(g))
    torch.cuda.synchronize()
    check_bins_exact(api, b, g, grids)


def test_bins_bit_exact_c64(api):
    """The 64^3 workload: 1-voxel Gaussians exactly on voxel centres put box bounds on
    integers, decided by the recipe's rounding."""
    w = inputs.workload("c64", with_data=False)
    grids = w.stacks + [w.volume]
    say("bins c64")
    b = api.Bins(w.gauss.n, grids)
    b.bin(api.GaussParams.from_host(w.gauss))
    torch.cuda.synchronize()
    check_bins_exact(api, b, w.gauss, grids)
    # the per-grid pair totals gm_bin hands back on the host equal the device array
    assert b.box_pairs_host == [b.pair_count(k) for k in range(len(grids))]


def render_ref(g, grids):
    return gauss.render_all(g, grids)


@pytest.mark.parametrize("seed", [0, 3])
def test_render_parity_ragged(api, seed):
    g, grids, _ = ragged_problem(seed)
    say("render ragged seed", seed)
    b = api.Bins(g.n, grids)
    b.bin(api.GaussParams.from_host(g))
    outs = api.render(b, list(range(len(grids))))
    torch.cuda.synchronize()
    refs = render_ref(g, grids)
    for k, (o, r) in enumerate(zip(outs, refs)):
        err = normwise(o.cpu().numpy(), r)
        say(f"  grid {k} normwise err {err:.3e}")
        assert err <= TOL


def test_render_deterministic_and_volume_entry(api):
    g, grids, _ = ragged_problem(5)
    b = api.Bins(g.n, grids)
    b.bin(api.GaussParams.from_host(g))
    a1 = api.render(b, [0, 1, 2, 3])
    a2 = api.render(b, [3, 1])
    v = api.render_volume(b, 3)
    torch.cuda.synchronize()
    assert torch.equal(a1[3], a2[0]) and torch.equal(a1[1], a2[1])
    assert torch.equal(a1[3], v)


def test_render_parity_c64(api):
    w = inputs.workload("c64", with_data=False)
    grids = w.stacks + [w.volume]
    say("render c64")
    b = api.Bins(w.gauss.n, grids)
    b.bin(api.GaussParams.from_host(w.gauss))
    outs = api.render(b, list(range(len(grids))))
    torch.cuda.synchronize()
    refs = render_ref(w.gauss, grids)
    for k, (o, r) in enumerate(zip(outs, refs)):
        err = normwise(o.cpu().numpy(), r)
        say(f"  grid {k} normwise err {err:.3e}")
        assert err <= TOL


def grads_gpu(api, g, grids, ids, dl, lam_aniso=0.0, lam_r=1.5):
    p = api.GaussParams.from_host(g)
    b = api.Bins(g.n, grids)
    b.bin(p)
    gr = api.GaussParams.zeros_like(p)
    dld = [torch.from_numpy(d).cuda() for d in dl]
    api.backward(p, b, ids, dld, gr, lam_aniso, lam_r)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in gr.tensors()], b


@pytest.mark.parametrize("seed", [0, 2])
def test_backward_parity_ragged(api, seed):
    g, grids, rng = ragged_problem(seed, n_g=400)
    dl = inputs.random_dl_di(grids, rng)
    say("backward ragged seed", seed)
    got, b = grads_gpu(api, g, grids, [0, 1, 2, 3], dl, 0.1, 1.5)
    ref = gauss.gradients(g, grids, dl, lam_aniso=0.1, lam_r=1.5)
    for name, a, r in zip(("mean", "quat", "log_scale", "logit"), got, ref):
        err = normwise(a, r)
        say(f"  {name} normwise err {err:.3e}")
        assert err <= TOL, name


def test_grid_partials_match_oracle(api):
    g, grids, rng = ragged_problem(4, n_g=300)
    dl = inputs.random_dl_di(grids, rng)
    _, b = grads_gpu(api, g, grids, [0, 1, 2, 3], dl)
    kappa = -0.5 / math.log(2.0)
    prep = gauss.prepare(g, grids)
    for k, (gr, (gt, lo, hi, ne, _)) in enumerate(zip(grids, prep)):
        d_amp, d_c, G_C = gauss.grid_partials(gr, gt, lo, hi, ne, dl[k])
        pg = b.grid_grads[k, :g.n].cpu().numpy().astype(np.float64)
        assert normwise(pg[:, 0], d_amp) <= TOL
        assert normwise(pg[:, 1:4], d_c) <= TOL
        dK = np.stack([G_C[:, 0, 0], G_C[:, 1, 1], G_C[:, 2, 2], G_C[:, 0, 1], G_C[:, 0, 2],
                       G_C[:, 1, 2]], 1) / kappa
        assert normwise(pg[:, 4:10], dK) <= TOL


def test_backward_stages_equal_backward(api):
    """gm_grid_partials followed by gm_chain gives gm_backward's result bit for bit, and the
    partials stage alone matches the oracle's grid-frame sums."""
    g, grids, rng = ragged_problem(5, n_g=400)
    dl = inputs.random_dl_di(grids, rng)
    ref, b = grads_gpu(api, g, grids, [0, 1, 2, 3], dl, 0.1, 1.5)
    p = api.GaussParams.from_host(g)
    b2 = api.Bins(p.n, grids)
    b2.bin(p)
    d_dl = [torch.from_numpy(d).cuda() for d in dl]
    api.grid_partials(p, b2, [0, 1, 2, 3], d_dl)
    torch.cuda.synchronize()
    assert torch.equal(b2.grid_grads, b.grid_grads)
    out = api.GaussParams.zeros_like(p)
    api.chain(p, b2, [0, 1, 2, 3], out, 0.1, 1.5)
    torch.cuda.synchronize()
    for a_, r_ in zip(out.tensors(), ref):
        assert np.array_equal(a_.cpu().numpy(), r_)


def test_backward_stacks_only_c64(api):
    w = inputs.workload("c64", with_data=False)
    rng = np.random.default_rng(77)
    dl = inputs.random_dl_di(w.stacks, rng)
    say("backward c64")
    got, _ = grads_gpu(api, w.gauss, w.stacks, [0, 1, 2], dl, 0.1, 1.5)
    ref = gauss.gradients(w.gauss, w.stacks, dl, lam_aniso=0.1, lam_r=1.5)
    # These Gaussians are isotropic, so the quaternion gradient is exactly zero in exact
    # arithmetic; both sides carry rounding noise only.  It is measured against the scale of
    # the covariance gradient it comes from (|dL/dq| <= 2 |G_Sigma| |Sigma| ~ |dL/ds|).
    scale = {"quat": np.max(np.abs(ref[2]))}
    for name, a, r in zip(("mean", "quat", "log_scale", "logit"), got, ref):
        s_ = max(np.max(np.abs(r)), scale.get(name, 0.0))
        err = np.max(np.abs(a - r)) / s_
        say(f"  {name} normwise err {err:.3e}")
        assert err <= TOL, name


def test_losses_and_adam(api):
    rng = np.random.default_rng(3)
    preds = [rng.normal(0, 1.2, size=(5, 7, 9)).astype(np.float32),
             rng.normal(0, 1.2, size=(3, 11, 13)).astype(np.float32)]
    targ = [rng.normal(size=p.shape).astype(np.float32) for p in preds]
    loss, dl = api.smooth_l1([torch.from_numpy(p).cuda() for p in preds],
                             [torch.from_numpy(t).cuda() for t in targ])
    rv, rg = gauss.smooth_l1(preds, targ)
    assert float(loss) == pytest.approx(rv, rel=1e-6)
    for a, r in zip(dl, rg):
        assert normwise(a.cpu().numpy(), r) <= 1e-6
    ls = rng.normal(-3, 0.6, size=(1000, 3)).astype(np.float32)
    g = inputs.Gaussians(np.zeros((1000, 3), np.float32), np.ones((1000, 4), np.float32), ls,
                         np.zeros(1000, np.float32))
    val = api.aniso(api.GaussParams.from_host(g), 1.5)
    assert float(val) == pytest.approx(gauss.aniso(ls, 1.5)[0], rel=1e-6)
    p0 = rng.normal(size=4097).astype(np.float32)
    m = np.zeros(4097)
    v = np.zeros(4097)
    pt, mt, vt = (torch.from_numpy(p0.copy()).cuda(), torch.zeros(4097, device="cuda"),
                  torch.zeros(4097, device="cuda"))
    p = p0.astype(np.float64)
    for step in range(1, 11):
        gr = rng.normal(size=4097).astype(np.float32)
        api.adam_step(pt, torch.from_numpy(gr).cuda(), mt, vt, 5e-3, step)
        p, m, v = gauss.adam(p, gr, m, v, step, 5e-3)
    # The update itself: both sides are fed the same float32 gradients, so p - p0 is pinned at
    # the FP32 bar of the update's size; the stored parameter is rounded to float32 once per
    # step (half a spacing of |p| each), which no bar relative to the update can absorb when
    # |p| is ~60x the update, so that rounding is allowed on top (10 steps, one spacing each).
    dp_gpu = pt.cpu().numpy().astype(np.float64) - p0
    dp_ref = p - p0
    spacing = np.spacing(np.maximum(np.abs(p0), np.abs(p)).astype(np.float32)).astype(np.float64)
    tol = TOL * np.max(np.abs(dp_ref)) + 10 * spacing
    assert np.all(np.abs(dp_gpu - dp_ref) <= tol), float(np.max(np.abs(dp_gpu - dp_ref) - tol))
    say(f"  Adam update max |dp_gpu - dp_ref| / max |dp_ref| = "
        f"{np.max(np.abs(dp_gpu - dp_ref)) / np.max(np.abs(dp_ref)):.2e}")
    # the moments, normwise
    assert normwise(mt.cpu().numpy(), m) <= TOL
    assert normwise(vt.cpu().numpy(), v) <= TOL
    a = rng.random(size=(9, 9, 9)).astype(np.float32)
    bb = rng.random(size=(9, 9, 9)).astype(np.float32)
    mse = api.mse(torch.from_numpy(a).cuda(), torch.from_numpy(bb).cuda())
    assert float(mse) == pytest.approx(np.mean((a.astype(np.float64) - bb) ** 2), rel=1e-6)


# ---- edge cases ---------------------------------------------------------------------------

def test_edge_empty_and_single(api):
    grids = [inputs.volume_grid(20), inputs.stack_grid("axial", 20, 5, 1.0)]
    for n in (0, 1):
        g = inputs.init_anisotropic(20, 1, np.random.default_rng(1)).subset(slice(0, n))
        p = api.GaussParams.from_host(g)
        b = api.Bins(n, grids)
        b.bin(p)
        check_bins_exact(api, b, g, grids)
        outs = api.render(b, [0, 1])
        refs = render_ref(g, grids)
        for o, r in zip(outs, refs):
            assert normwise(o.cpu().numpy(), r) <= TOL
        gr = api.GaussParams.zeros_like(p)
        api.backward(p, b, [0, 1], [torch.ones(gg.shape, device="cuda") for gg in grids], gr)
        torch.cuda.synchronize()


def test_edge_outside_face_and_one_tile(api):
    n = 33
    rng = np.random.default_rng(12)
    g = inputs.init_anisotropic(n, 64, rng)
    g.mean[:8] = np.float32(3.0)                        # far outside
    g.mean[8:16, 0] = np.float32(1.0)                   # on the +x face
    g.mean[16:24, 1] = np.float32(-1.0)                 # on the -y face
    g.mean[24:] = np.float32(-0.9)                      # all near one corner tile
    g.log_scale[24:] = np.float32(math.log(0.5 * 2 / n))
    grids = [inputs.volume_grid(n), inputs.stack_grid("coronal", n, 8, 1.0)]
    b = api.Bins(g.n, grids)
    b.bin(api.GaussParams.from_host(g))
    check_bins_exact(api, b, g, grids)
    outs = api.render(b, [0, 1])
    for o, r in zip(outs, render_ref(g, grids)):
        assert normwise(o.cpu().numpy(), r) <= TOL


def test_edge_crowded_tile_many_sort_blocks(api):
    """Twenty thousand Gaussians crowded into the tiles at one corner: tens of thousands of
    entries share a handful of keys, so one digit holds whole sort blocks (4096 keys) and the
    equal keys must keep ascending Gaussian order across blocks, in both passes (320 tiles:
    9-bit keys)."""
    n = 64
    rng = np.random.default_rng(21)
    g = inputs.init_anisotropic(n, 20500, rng)
    g.mean[:20000] = (np.float32(-0.9) + rng.uniform(-0.01, 0.01, size=(20000, 3))).astype(np.float32)
    g.log_scale[:20000] = np.float32(math.log(0.5 * 2 / n))
    grids = [inputs.volume_grid(n), inputs.stack_grid("axial", n, 16, 1.0)]
    say("crowded tile, sort blocks")
    b = api.Bins(g.n, grids)
    b.bin(api.GaussParams.from_host(g))
    torch.cuda.synchronize()
    assert b.n_pairs > 4 * 4096
    check_bins_exact(api, b, g, grids)


def test_edge_huge_gaussian_and_capacity_growth(api):
    n = 24
    g = inputs.init_anisotropic(n, 50, np.random.default_rng(2))
    g.log_scale[0] = np.float32(math.log(6.0 * 2 / n))   # box covers most of the grid
    grids = [inputs.volume_grid(n)]
    b = api.Bins(g.n, grids, capacity=16)                # forces GM_ERR_CAPACITY then retry
    b.bin(api.GaussParams.from_host(g))
    assert b.capacity >= b.n_pairs
    check_bins_exact(api, b, g, grids)
    out = api.render(b, [0])[0]
    assert normwise(out.cpu().numpy(), render_ref(g, grids)[0]) <= TOL


def test_edge_capacity_error_reported(api):
    from paper_2603_00145_amd import _lib
    import ctypes
    g = inputs.init_anisotropic(16, 40, np.random.default_rng(3))
    grids = [inputs.volume_grid(16)]
    b = api.Bins(g.n, grids, capacity=4)
    p = api.GaussParams.from_host(g)
    npairs = ctypes.c_int64()
    st = _lib.load().gm_bin(ctypes.byref(p.struct()), b._cgrids, 1,
                            ctypes.byref(_lib.GmBinOpts(3.0)), ctypes.byref(b.struct()),
                            ctypes.byref(npairs), api._stream())
    assert st == _lib.GM_ERR_CAPACITY and npairs.value > 4
    with pytest.raises(_lib.GmError):
        api.render(b, [0])


def test_edge_nonfinite_reported(api):
    from paper_2603_00145_amd import _lib
    g = inputs.init_anisotropic(16, 10, np.random.default_rng(4))
    g.quat[3] = 0
    g.mean[5, 1] = np.nan
    b = api.Bins(g.n, [inputs.volume_grid(16)])
    with pytest.raises(_lib.GmError) as ei:
        b.bin(api.GaussParams.from_host(g))
    assert ei.value.status == _lib.GM_ERR_NONFINITE
    b.bin(api.GaussParams.from_host(g), allow_nonfinite=True)
    glo, ghi = (t.cpu().numpy() for t in b.boxes(0))
    assert not (glo[3] <= ghi[3]).all() and not (glo[5] <= ghi[5]).all()


def test_invalid_arguments_rejected(api):
    from paper_2603_00145_amd import _lib
    import ctypes
    bad = inputs.Grid(0, 4, 4, np.eye(3, 4))
    with pytest.raises(_lib.GmError):
        api.Bins(4, [bad])
    with pytest.raises(_lib.GmError):
        api.adam_step(*(torch.zeros(4, device="cuda") for _ in range(4)), lr=1e-3, step=0)

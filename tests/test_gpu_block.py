"""The paper's block-radius query (Eqs. 4-6) on the GPU: boxes, tile counts and pair totals
bit-exact against the oracle on the 64^3 workload's axis-aligned stacks and volume, voxel
values at sampled voxels; on rotated stacks (voxel sets that are not boxes, tested voxel by
voxel) every voxel's value and every Gaussian's grid-frame partials against the oracle's
brute-force sums over the same sets, the fused render + field + loss against its parts, and
reconstructions running on both."""
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
def mods():
    from paper_2603_00145_amd import _lib, api
    api.load()
    return _lib, api


@pytest.mark.parametrize("res,r", [(32, 1), (32, 3), (20, 2), (48, 1)])
def test_block_boxes_and_values(mods, res, r):
    _lib, api = mods
    w = inputs.workload("c64", with_data=False)
    g = w.gauss
    grids = list(w.stacks) + [w.volume]
    p = api.GaussParams.from_host(g)
    b = api.Bins(p.n, grids, block_radius=r, cell_resolution=res)
    b.bin(p)
    tile = _lib.tile_dims()
    rng = np.random.default_rng(res * 10 + r)
    outs = api.render(b, list(range(len(grids))))
    mean, quat, ls, logit = gauss.params64(g)
    for k, grid in enumerate(grids):
        lo, hi, ne, _ = recipe.block_boxes(g.mean, g.quat, g.log_scale, g.logit, grid, res, r)
        glo, ghi = (t.cpu().numpy() for t in b.boxes(k))
        gne = (glo <= ghi).all(1)
        assert np.array_equal(gne, ne), grid.name
        assert np.array_equal(glo[ne], lo[ne]) and np.array_equal(ghi[ne], hi[ne]), grid.name
        counts = recipe.tile_counts(lo, hi, ne, tile)
        assert np.array_equal(b.tile_count[k, :p.n].cpu().numpy(), counts), grid.name
        assert b.box_pairs_host[k] == int(recipe.box_volume(lo, hi, ne).sum()), grid.name
        gt = gauss.grid_terms(mean, quat, ls, logit, grid)
        pts = np.stack([rng.integers(0, d, 400) for d in (grid.nx, grid.ny, grid.nz)], 1)
        ref = gauss.render_points(pts, gt, lo, hi, ne)
        got = outs[k].cpu().numpy()[pts[:, 2], pts[:, 1], pts[:, 0]]
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        say(f"  res {res} r {r} {grid.name}: boxes exact, {b.box_pairs_host[k]} pairs, "
            f"values normwise {err:.2e}")
        assert err <= TOL


def normwise(a, r):
    r = np.asarray(r, np.float64)
    return np.max(np.abs(np.asarray(a, np.float64) - r)) / max(np.max(np.abs(r)), 1e-30)


def rotated_problem(rng, n=41, n_g=900):
    """Two rotated stacks (2 and 20 degrees; ragged tiles), an unrotated stack and the volume:
    one launch holds masked and unmasked grids."""
    g = inputs.init_anisotropic(n, n_g, rng)
    grids = [inputs.stack_grid("axial", n, 11, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("coronal", 30, 7, 1.0, *inputs.random_rigid(rng, 20, 2, 30)),
             inputs.stack_grid("sagittal", n, 9, 1.0),
             inputs.volume_grid(n)]
    return g, grids


@pytest.mark.parametrize("res,r", [(12, 1), (24, 2), (40, 1), (1, 1), (7, 9)])
def test_block_query_on_rotated_grids(mods, res, r):
    """(1, 1): one cell, every voxel of every grid in every block; (7, 9): blocks wider than
    the cell grid.  A tenth of the Gaussians sit outside [-1, 1]^3 (negative or beyond-last
    cells)."""
    _lib, api = mods
    rng = np.random.default_rng(100 + res + r)
    g, grids = rotated_problem(rng)
    out = rng.choice(g.n, g.n // 10, replace=False)
    g.mean[out] = rng.uniform(-1.3, 1.3, (len(out), 3)).astype(np.float32)
    ids = list(range(len(grids)))
    say(f"block query on rotated grids: res {res} r {r}")
    p = api.GaussParams.from_host(g)
    b = api.Bins(p.n, grids, block_radius=r, cell_resolution=res)
    b.bin(p)
    outs = api.render(b, ids)
    dl = inputs.random_dl_di(grids, rng)
    api.grid_partials(p, b, ids, [torch.from_numpy(d).cuda() for d in dl])
    torch.cuda.synchronize()
    mean, quat, ls, logit = gauss.params64(g)
    gcell = recipe.mean_cells(g.mean, res)
    kappa = -0.5 / np.log(2.0)
    for k, grid in enumerate(grids):
        gt = gauss.grid_terms(mean, quat, ls, logit, grid)
        aligned = recipe.world_axes(grid) is not None
        if aligned:
            lo, hi, ne, _ = recipe.block_boxes(g.mean, g.quat, g.log_scale, g.logit, grid, res, r)
            ref = gauss.render(grid, gt, lo, hi, ne)
            d_amp, d_c, G_C = gauss.grid_partials(grid, gt, lo, hi, ne, dl[k])
        else:
            _, _, _, valid = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, grid)
            vcell = recipe.voxel_cells(grid, res)
            ref = gauss.render_cells(grid, gt, vcell, gcell, valid, r)
            d_amp, d_c, G_C = gauss.grid_partials_cells(grid, gt, vcell, gcell, valid, r, dl[k])
            # the GPU machine holds every voxel of the set
            glo, ghi = (t.cpu().numpy() for t in b.boxes(k))
            z, y, x = np.meshgrid(np.arange(grid.nz), np.arange(grid.ny), np.arange(grid.nx),
                                  indexing="ij")
            vox = np.stack([x, y, z], -1).reshape(-1, 3)
            member = (np.abs(vcell[None, :, :] - gcell[:, None, :]) <= r).all(2) & valid[:, None]
            for i in np.flatnonzero(member.any(1)):
                v = vox[member[i]]
                assert (v >= glo[i]).all() and (v <= ghi[i]).all(), (grid.name, i)
        err = normwise(outs[k].cpu().numpy(), ref)
        pg = b.grid_grads[k, :g.n].cpu().numpy().astype(np.float64)
        dK = np.stack([G_C[:, 0, 0], G_C[:, 1, 1], G_C[:, 2, 2], G_C[:, 0, 1], G_C[:, 0, 2],
                       G_C[:, 1, 2]], 1) / kappa
        e_p = [normwise(pg[:, 0], d_amp), normwise(pg[:, 1:4], d_c), normwise(pg[:, 4:10], dK)]
        say(f"  {grid.name} ({'aligned' if aligned else 'rotated'}): values {err:.2e}, "
            f"partials {max(e_p):.2e}")
        assert err <= TOL, grid.name
        assert max(e_p) <= TOL, grid.name


def test_block_query_on_the_rotated_128_stacks(mods):
    """The full 128^3 workload (200k Gaussians, three 128x128x32 stacks rotated by up to 2
    degrees) under the block query: 600 sampled voxels per stack against the oracle's
    brute-force sum over every Gaussian with the cell test, and the grid-frame partials of 400
    sampled Gaussians per stack against the oracle's sums over every voxel of the stack."""
    _lib, api = mods
    res, r = 64, 2
    w = inputs.workload("c128", with_data=False)
    g = w.gauss
    p = api.GaussParams.from_host(g)
    b = api.Bins(p.n, w.stacks, block_radius=r, cell_resolution=res)
    b.bin(p)
    outs = api.render(b, list(range(len(w.stacks))))
    rng = np.random.default_rng(128)
    dl = inputs.random_dl_di(w.stacks, rng)
    api.grid_partials(p, b, list(range(len(w.stacks))), [torch.from_numpy(d).cuda() for d in dl])
    torch.cuda.synchronize()
    mean, quat, ls, logit = gauss.params64(g)
    gcell = recipe.mean_cells(g.mean, res)
    kappa = -0.5 / np.log(2.0)
    for k, grid in enumerate(w.stacks):
        assert recipe.world_axes(grid) is None          # rotated: the masked path
        gt = gauss.grid_terms(mean, quat, ls, logit, grid)
        _, _, _, valid = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, grid)
        sel = rng.choice(grid.n_voxels, 600, replace=False)
        z, rem = np.divmod(sel, grid.nx * grid.ny)
        y, x = np.divmod(rem, grid.nx)
        pcell = recipe.voxel_cells(grid, res)[sel]
        ref = gauss.render_points_cells(np.stack([x, y, z], 1), pcell, gt, gcell, valid, r)
        got = outs[k].cpu().numpy().reshape(-1)[sel]
        err = normwise(got, ref)
        # partials of sampled Gaussians whose block reaches the stack
        sub = np.sort(rng.choice(g.n, 400, replace=False))
        gs = {key: (v[sub] if isinstance(v, np.ndarray) and v.shape[:1] == (g.n,) else v)
              for key, v in gt.items()}
        vcell = recipe.voxel_cells(grid, res)
        d_amp, d_c, G_C = gauss.grid_partials_cells(grid, gs, vcell, gcell[sub], valid[sub], r,
                                                    dl[k])
        pg = b.grid_grads[k, sub].cpu().numpy().astype(np.float64)
        dK = np.stack([G_C[:, 0, 0], G_C[:, 1, 1], G_C[:, 2, 2], G_C[:, 0, 1], G_C[:, 0, 2],
                       G_C[:, 1, 2]], 1) / kappa
        e_p = max(normwise(pg[:, 0], d_amp), normwise(pg[:, 1:4], d_c), normwise(pg[:, 4:10], dK))
        say(f"  c128 {grid.name}, block r={r} res={res}: {b.box_pairs_host[k]} box pairs, "
            f"sampled values normwise {err:.2e}, sampled partials {e_p:.2e}")
        assert err <= TOL, grid.name
        assert e_p <= TOL, grid.name


def test_fused_render_field_loss_on_rotated_block_query(mods):
    """The masked form of the fused render + field + loss against the render, the field's
    forward and the loss called one after the other (bit for bit; the loss to 1e-6)."""
    _lib, api = mods
    from paper_2603_00145_amd import nrf
    rng = np.random.default_rng(5)
    g, grids = rotated_problem(rng, n_g=600)
    ids = list(range(len(grids)))
    say("fused render + field + loss, block query on rotated grids")
    targ = [torch.from_numpy(rng.normal(0.3, 1.0, size=gr.shape).astype(np.float32)).cuda()
            for gr in grids]
    b = api.Bins(g.n, grids, block_radius=2, cell_resolution=20)
    b.bin(api.GaussParams.from_host(g))
    net = nrf.NRF(n_freq=16, depth=3, seed=3, zero_last=False)
    outs = api.render(b, ids)
    for k in ids:
        net.forward_add(grids[k], outs[k])
    ref_loss, ref_dl = api.smooth_l1(outs, targ)
    stored = [torch.full(gr.shape, float("nan"), device="cuda") for gr in grids]
    loss, dl = api.render_loss(b, ids, targ, outs=stored, nrf=net)
    torch.cuda.synchronize()
    for k in ids:
        assert torch.equal(stored[k], outs[k]), f"grid {k}: rendering + field differs"
        assert torch.equal(dl[k], ref_dl[k]), f"grid {k}: dL/dI differs"
    assert float(loss) == pytest.approx(float(ref_loss), rel=1e-6)


def test_reconstruction_with_block_query_on_rotated_stacks(mods):
    _lib, api = mods
    from paper_2603_00145_amd import recon
    w = inputs.workload("small", device="cuda")           # stacks with rigid offsets
    data = [torch.as_tensor(d) for d in w.stack_data]
    cfg = recon.TrainConfig(n_iter=40, block_radius=2, cell_resolution=12)
    r = recon.Reconstruction(w.stacks, data, api.devox_init(12, w.stacks, data), cfg, w.volume,
                             w.phantom)
    hist = r.run()
    say(f"  rotated stacks, block r=2 psnr {hist[0]['psnr']:.2f} -> {hist[-1]['psnr']:.2f}")
    assert hist[-1]["psnr"] > hist[0]["psnr"]


def test_reconstruction_with_block_query(mods):
    _lib, api = mods
    from paper_2603_00145_amd import recon
    w = inputs.workload("c64", device="cuda")
    data = [torch.as_tensor(d) for d in w.stack_data]
    cfg = recon.TrainConfig(n_iter=40, block_radius=3, cell_resolution=24)
    r = recon.Reconstruction(w.stacks, data, api.devox_init(24, w.stacks, data), cfg, w.volume,
                             w.phantom)
    hist = r.run()
    say(f"  block r=3 psnr {hist[0]['psnr']:.2f} -> {hist[-1]['psnr']:.2f}")
    assert hist[-1]["psnr"] > hist[0]["psnr"]

"""Pins of the oracle's block-radius query (Sec. 3.3.1, Eqs. 4-6): every voxel tested one by
one, the closed form when cells are whole voxel pairs, radius monotonicity and coverage."""
import numpy as np
import pytest

from oracle import recipe
from paper_2603_00145_amd import inputs


def gaussians(n, rng, spread=1.1):
    mean = rng.uniform(-spread, spread, (n, 3)).astype(np.float32)
    quat = rng.normal(size=(n, 4)).astype(np.float32)
    ls = rng.normal(-3, 0.3, (n, 3)).astype(np.float32)
    logit = rng.normal(size=n).astype(np.float32)
    return mean, quat, ls, logit


def literal(mean, grid, res, r):
    """Per voxel: x = index->world of the axis-aligned grid, Eq. 4 cells, Eq. 5 test."""
    A = np.asarray(grid.world_to_index, np.float64)
    axes = recipe.world_axes(grid)
    dims = [grid.nx, grid.ny, grid.nz]
    out = []
    for mu in mean.astype(np.float64):
        box = []
        for j in range(3):
            a = axes[j]
            ins = [v for v in range(dims[j])
                   if abs(recipe.cell_of((v - A[j, 3]) / A[j, a], res) - recipe.cell_of(mu[a], res)) <= r]
            box.append((min(ins), max(ins)) if ins else None)
        out.append(box)
    return out


@pytest.mark.parametrize("res,r", [(16, 1), (32, 2), (10, 3), (7, 0)])
def test_block_boxes_match_voxel_by_voxel(res, r):
    rng = np.random.default_rng(res + r)
    mean, quat, ls, logit = gaussians(60, rng)
    grids = [inputs.volume_grid(24), inputs.stack_grid("coronal", 20, 6, 1.0),
             inputs.stack_grid("sagittal", 18, 5, 1.0)]
    for grid in grids:
        lo, hi, ne, valid = recipe.block_boxes(mean, quat, ls, logit, grid, res, r)
        ref = literal(mean, grid, res, r)
        for i, box in enumerate(ref):
            if any(b is None for b in box):
                assert not ne[i]
            else:
                assert ne[i]
                assert [tuple(x) for x in zip(lo[i], hi[i])] == box, (grid.name, i)


def test_closed_form_two_voxels_per_cell():
    # volume of n = 2 res voxels: cell k covers voxels 2k and 2k + 1 on every axis
    res, r, n = 16, 2, 32
    rng = np.random.default_rng(0)
    mean, quat, ls, logit = gaussians(200, rng, spread=0.99)
    lo, hi, ne, _ = recipe.block_boxes(mean, quat, ls, logit, inputs.volume_grid(n), res, r)
    cell = np.floor((mean.astype(np.float64) + 1.0) * res / 2.0)
    np.testing.assert_array_equal(lo, np.clip(2 * (cell - r), 0, n - 1))
    np.testing.assert_array_equal(hi, np.clip(2 * (cell + r) + 1, 0, n - 1))
    assert ne.all()


def test_radius_monotone_and_full_coverage():
    rng = np.random.default_rng(1)
    mean, quat, ls, logit = gaussians(50, rng, spread=0.9)
    grid = inputs.stack_grid("axial", 20, 6, 1.0)
    prev = None
    for r in range(0, 5):
        lo, hi, ne, _ = recipe.block_boxes(mean, quat, ls, logit, grid, 12, r)
        if prev is not None:
            assert (lo <= prev[0]).all() and (hi >= prev[1]).all()
        prev = (lo, hi)
    lo, hi, ne, _ = recipe.block_boxes(mean, quat, ls, logit, grid, 12, 12)
    assert (lo == 0).all() and (hi == np.array([19, 19, 5])).all()


def test_rotated_grid_rejected():
    rng = np.random.default_rng(2)
    mean, quat, ls, logit = gaussians(4, rng)
    g = inputs.stack_grid("axial", 16, 4, 1.0, *inputs.random_rigid(rng, 2.0, 1.0, 16))
    with pytest.raises(ValueError):
        recipe.block_boxes(mean, quat, ls, logit, g, 8, 2)


def cell_sets(vcell, gcell, valid, r):
    """Per Gaussian: the voxels (storage-order indices) the block query gives it."""
    return [np.flatnonzero((np.abs(vcell - gcell[i]) <= r).all(1)) if valid[i] else
            np.zeros(0, np.int64) for i in range(gcell.shape[0])]


@pytest.mark.parametrize("res,r", [(16, 1), (10, 2)])
def test_cell_sets_are_the_boxes_on_exact_axis_aligned_grids(res, r):
    """On unrotated grids with power-of-two sizes both routes to a voxel's world position
    (the per-axis division of block_boxes, the index->world affine of voxel_cells) are exact,
    so the cell test must select exactly block_boxes' boxes, and the brute-force sums over
    those sets must equal the box sums bit for bit."""
    from oracle import gauss
    rng = np.random.default_rng(40 + r)
    mean, quat, ls, logit = gaussians(40, rng, spread=1.05)
    grids = [inputs.volume_grid(16), inputs.stack_grid("coronal", 32, 8, 1.0),
             inputs.stack_grid("sagittal", 16, 4, 1.0)]
    for grid in grids:
        lo, hi, ne, valid = recipe.block_boxes(mean, quat, ls, logit, grid, res, r)
        vcell = recipe.voxel_cells(grid, res)
        gcell = recipe.mean_cells(mean, res)
        sets = cell_sets(vcell, gcell, valid, r)
        z, y, x = np.meshgrid(np.arange(grid.nz), np.arange(grid.ny), np.arange(grid.nx),
                              indexing="ij")
        vox = np.stack([x, y, z], -1).reshape(-1, 3)
        for i in range(len(sets)):
            inbox = ((vox >= lo[i]) & (vox <= hi[i])).all(1) & bool(ne[i])
            np.testing.assert_array_equal(sets[i], np.flatnonzero(inbox), err_msg=f"{grid.name} {i}")
        g = inputs.Gaussians(mean, quat, ls, logit)
        (gt, _, _, _, _), = gauss.prepare(g, [grid])
        a = gauss.render_cells(grid, gt, vcell, gcell, valid, r)
        b = gauss.render(grid, gt, lo, hi, ne)
        np.testing.assert_array_equal(a, b)
        dl = rng.normal(size=grid.shape)
        pa = gauss.grid_partials_cells(grid, gt, vcell, gcell, valid, r, dl)
        pb = gauss.grid_partials(grid, gt, lo, hi, ne, dl)
        for u, w in zip(pa, pb):
            np.testing.assert_array_equal(u, w)


def test_voxel_cells_on_a_rotated_grid_follow_the_world_position():
    """On a rotated, shifted stack the cell of every voxel is that of its world position
    found another way (solving L x = v - t by LU), except within 1e-9 of a cell boundary; and
    the cell test is the world interval [2 (c - r) / res - 1, 2 (c + r + 1) / res - 1) of
    each axis (Eqs. 4-5 solved for x)."""
    rng = np.random.default_rng(7)
    res, r = 12, 1
    grid = inputs.stack_grid("axial", 24, 6, 1.0, *inputs.random_rigid(rng, 25.0, 2.0, 24))
    vcell = recipe.voxel_cells(grid, res)
    A = np.asarray(grid.world_to_index, np.float64)
    z, y, x = np.meshgrid(np.arange(grid.nz), np.arange(grid.ny), np.arange(grid.nx),
                          indexing="ij")
    vox = np.stack([x, y, z], -1).reshape(-1, 3).astype(np.float64)
    xw = np.linalg.solve(A[:, :3], (vox - A[:, 3]).T).T
    u = (xw + 1.0) * res / 2.0
    near = np.abs(u - np.rint(u)) < 1e-9
    ok = (vcell == np.floor(u)) | near
    assert ok.all()
    assert (~near).mean() > 0.99
    mean = rng.uniform(-0.9, 0.9, (30, 3)).astype(np.float32)
    gcell = recipe.mean_cells(mean, res)
    sets = cell_sets(vcell, gcell, np.ones(30, bool), r)
    for i in range(30):
        lo_w = 2.0 * (gcell[i] - r) / res - 1.0
        hi_w = 2.0 * (gcell[i] + r + 1) / res - 1.0
        inside = ((xw >= lo_w - 1e-9) & (xw < hi_w + 1e-9)).all(1)
        strict = ((xw >= lo_w + 1e-9) & (xw < hi_w - 1e-9)).all(1)
        member = np.zeros(len(vox), bool)
        member[sets[i]] = True
        assert (member <= inside).all() and (strict <= member).all()
        assert member.any()


def test_point_sums_with_the_cell_test_equal_the_grid_sums():
    """The point form of the cell-test sum gives the grid form's values at those voxels."""
    from oracle import gauss
    rng = np.random.default_rng(9)
    res, r = 12, 1
    grid = inputs.stack_grid("coronal", 20, 5, 1.0, *inputs.random_rigid(rng, 15.0, 1.0, 20))
    mean, quat, ls, logit = gaussians(50, rng, spread=0.9)
    g = inputs.Gaussians(mean, quat, ls, logit)
    (gt, _, _, _, valid), = gauss.prepare(g, [grid])
    vcell = recipe.voxel_cells(grid, res)
    gcell = recipe.mean_cells(mean, res)
    full = gauss.render_cells(grid, gt, vcell, gcell, valid, r).reshape(-1)
    sel = rng.choice(grid.n_voxels, 200, replace=False)
    z, rem = np.divmod(sel, grid.nx * grid.ny)
    y, x = np.divmod(rem, grid.nx)
    pts = np.stack([x, y, z], 1)
    got = gauss.render_points_cells(pts, vcell[sel], gt, gcell, valid, r)
    np.testing.assert_array_equal(got, full[sel])

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

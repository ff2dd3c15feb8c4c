"""Pins of the oracle's gradient with respect to a grid's world->index affine (the quantity the
joint optimisation of the stacks' rigid transforms T_k, Sec. 3.3.2, needs): complex-step and
central differences of the numpy renderer with boxes held fixed, and the translation column as
the sum of the centre partials."""
import numpy as np
import pytest

from oracle import gauss, recipe
from paper_2603_00145_amd import inputs


def problem(seed):
    rng = np.random.default_rng(seed)
    n = 10
    g = inputs.init_anisotropic(n, 5, rng)
    g.log_scale += np.float32(0.5)
    grids = [inputs.stack_grid("axial", n, 4, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("coronal", n, 3, 1.0),
             inputs.volume_grid(n)]
    dl = inputs.random_dl_di(grids, rng)
    return g, grids, dl


def objective(g, grid, dl, A):
    """sum_v dl[v] I[v] on ``grid`` with its affine replaced by A (possibly complex), boxes
    fixed at the real grid."""
    mean, quat, ls, logit = gauss.params64(g)
    lo, hi, ne, _ = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, grid)
    shim = inputs.Grid(grid.nx, grid.ny, grid.nz, A, grid.psf_sigma_z)
    gt = gauss.grid_terms(mean, quat, ls, logit, shim)
    return (gauss.render_numpy(grid, gt, lo, hi, ne) * dl).sum()


def analytic(g, grid, dl):
    mean, quat, ls, logit = gauss.params64(g)
    (gt, lo, hi, ne, _), = gauss.prepare(g, [grid])
    part = gauss.grid_partials(grid, gt, lo, hi, ne, dl)
    return gauss.pose_grad(mean, quat, ls, logit, grid, part), part


@pytest.mark.parametrize("seed", [0, 1])
def test_pose_gradient_vs_complex_step(seed):
    g, grids, dl = problem(seed)
    for grid, d in zip(grids, dl):
        ana, _ = analytic(g, grid, d)
        A0 = np.asarray(grid.world_to_index, np.float64)
        cs = np.zeros((3, 4))
        h = 1e-30
        for idx in np.ndindex(3, 4):
            A = A0.astype(np.complex128)
            A[idx] += 1j * h
            cs[idx] = objective(g, grid, d, A).imag / h
        err = np.max(np.abs(ana - cs)) / np.max(np.abs(cs))
        assert err < 1e-10, (grid.name, err)


def test_pose_gradient_vs_central_differences():
    g, grids, dl = problem(2)
    grid, d = grids[0], dl[0]
    ana, _ = analytic(g, grid, d)
    A0 = np.asarray(grid.world_to_index, np.float64)
    for idx in np.ndindex(3, 4):
        h = 1e-6 * max(1.0, abs(A0[idx]))
        Ap, Am = A0.copy(), A0.copy()
        Ap[idx] += h
        Am[idx] -= h
        fd = (objective(g, grid, d, Ap) - objective(g, grid, d, Am)) / (2 * h)
        assert abs(ana[idx] - fd) <= 1e-6 * np.max(np.abs(ana)), idx


def test_translation_column_is_sum_of_centre_partials():
    g, grids, dl = problem(3)
    ana, (d_amp, d_c, G_C) = analytic(g, grids[1], dl[1])
    np.testing.assert_allclose(ana[:, 3], d_c.sum(0), rtol=1e-14)

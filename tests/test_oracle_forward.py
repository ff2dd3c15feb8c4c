"""Pins of the oracle's forward definitions against closed forms, quadrature, invariants and
brute force (CPU only)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import gauss, recipe
from paper_2603_00145_amd import inputs


def one(mean, quat, log_scale, logit):
    return inputs.Gaussians(np.asarray([mean], np.float32), np.asarray([quat], np.float32),
                            np.asarray([log_scale], np.float32),
                            np.asarray(logit, np.float32).reshape(1))


def vox_world(i, n):
    return -1.0 + (2.0 * i + 1.0) / n


def test_exp_recipe_matches_libm():
    x = np.concatenate([np.linspace(-30, 30, 20001), [0.0, -0.0, 1e-300, 0.5 * math.log(2)]])
    got = recipe.exp_recipe(x)
    ref = np.exp(x)
    assert np.max(np.abs(got - ref) / ref) < 4e-16


def test_parameter_count_is_eleven():
    # Eq. 2-3: centre 3 + quaternion 4 + log-scale 3 + intensity 1 = 11 floats; 59/11 ~ 5.4
    g = inputs.init_isotropic(16, 5, np.random.default_rng(0))
    per = g.mean.shape[1] + g.quat.shape[1] + g.log_scale.shape[1] + 1
    assert per == 11
    assert round(59 / per, 1) == 5.4


def test_centre_value_is_alpha():
    n = 17
    grid = inputs.volume_grid(n)
    g = one([vox_world(8, n)] * 3, [1, 0, 0, 0], [math.log(1.3 * 2 / n)] * 3, [0.7])
    (gt, lo, hi, ne, _), = gauss.prepare(g, [grid])
    out = gauss.render(grid, gt, lo, hi, ne)
    alpha = 1 / (1 + math.exp(-float(np.float32(0.7))))
    assert out[8, 8, 8] == pytest.approx(alpha, rel=1e-14)


def test_identity_rotation_is_separable():
    n = 20
    grid = inputs.volume_grid(n)
    sig_vox = np.array([0.9, 1.7, 1.25])
    mu_idx = np.array([9.3, 10.1, 8.7])
    g = one(vox_world(mu_idx, n), [2.0, 0, 0, 0], np.log(sig_vox * 2 / n), [-0.3])
    (gt, lo, hi, ne, _), = gauss.prepare(g, [grid])
    out = gauss.render(grid, gt, lo, hi, ne)
    # recompute in float64 from the float32 stored parameters
    mu_idx = (g.mean[0].astype(np.float64) + 1) * n / 2 - 0.5
    sig = np.exp(g.log_scale[0].astype(np.float64)) * n / 2
    alpha = 1 / (1 + math.exp(-float(g.logit[0])))
    for (x, y, z) in [(9, 10, 8), (11, 12, 9), (8, 7, 10), (lo[0, 0], lo[0, 1], lo[0, 2])]:
        d = np.array([x, y, z]) - mu_idx
        ref = alpha * np.prod(np.exp(-0.5 * (d / sig) ** 2))
        assert out[z, y, x] == pytest.approx(ref, rel=1e-13)


def test_quaternion_90deg_about_z_swaps_xy_scales():
    n = 24
    grid = inputs.volume_grid(n)
    c = vox_world(np.array([11.2, 12.4, 11.7]), n)
    sx, sy, sz = 0.8, 2.1, 1.4
    ls = np.log(np.array([sx, sy, sz]) * 2 / n)
    h = math.sqrt(0.5)
    a = one(c, [h, 0, 0, h], ls, [0.4])
    b = one(c, [1, 0, 0, 0], ls[[1, 0, 2]], [0.4])
    ga = gauss.prepare(a, [grid], cutoff=6.0)[0][0]
    gb = gauss.prepare(b, [grid], cutoff=6.0)[0][0]
    # the Hamilton matrix of a +90 deg turn about z maps e_x to e_y
    R = gauss.quat_to_rot(np.array([[h, 0, 0, h]]))[0]
    assert np.allclose(R @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    assert np.allclose(ga["C"], gb["C"], rtol=1e-6, atol=1e-9)


def test_untruncated_mass_closed_form_volume_and_stack():
    """sum_v I[v] = alpha (2 pi)^{3/2} sqrt(det Sigma_idx) for a Gaussian far from the grid
    faces with sigma >= 1.5 voxels (lattice-sum error < 1e-12), on a volume grid and on a
    stack grid (the slice profile preserves mass)."""
    n = 48
    rng = np.random.default_rng(3)
    q = rng.normal(size=4)
    g = one(vox_world(np.array([23.3, 24.6, 23.9]), n), q,
            np.log(np.array([1.8, 2.4, 3.0]) * 2 / n), [1.1])
    alpha = 1 / (1 + math.exp(-float(g.logit[0])))
    vol = inputs.volume_grid(n)
    stk = inputs.stack_grid("axial", n, n // 2, fwhm_slices=1.0)
    for grid in (vol, stk):
        (gt, lo, hi, ne, _), = gauss.prepare(g, [grid], cutoff=9.0)
        out = gauss.render(grid, gt, lo, hi, ne)
        ref = alpha * (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(gt["Sig_idx"][0]))
        assert out.sum() == pytest.approx(ref, rel=1e-9)


def test_slice_profile_closed_form_against_quadrature():
    """A stack voxel's value equals the volume model integrated along the slice normal with
    the normalised Gaussian profile (numerical quadrature)."""
    n = 32
    rng = np.random.default_rng(5)
    g = one(vox_world(np.array([15.2, 16.7, 14.1]), n), rng.normal(size=4),
            np.log(np.array([1.1, 0.7, 1.6]) * 2 / n), [0.2])
    R_off, sh = inputs.random_rigid(rng, 2.0, 1.0, n)
    stk = inputs.stack_grid("coronal", n, n // 4, fwhm_slices=1.0, rigid=R_off, shift=sh)
    (gt, lo, hi, ne, _), = gauss.prepare(g, [stk], cutoff=12.0)
    mean, quat, ls, logit = gauss.params64(g)
    wt = gauss.world_terms(mean, quat, ls, logit)
    Sinv = np.linalg.inv(wt["Sigma"][0])
    alpha = wt["alpha"][0]
    Ai = stk.index_to_world()
    sig = stk.psf_sigma_z
    out = gauss.render(stk, gt, lo, hi, ne)

    def model(xw):
        d = xw - mean[0]
        return alpha * math.exp(-0.5 * d @ Sinv @ d)

    cidx = gt["c"][0]
    for v in [np.rint(cidx).astype(int), np.rint(cidx).astype(int) + [1, -1, 0],
              np.rint(cidx).astype(int) + [0, 1, 1]]:
        def f(u):
            p = v.astype(np.float64) + np.array([0, 0, u])
            xw = Ai[:, :3] @ p + Ai[:, 3]
            return model(xw) * math.exp(-0.5 * (u / sig) ** 2) / (sig * math.sqrt(2 * math.pi))
        ref, _ = integrate.quad(f, -12 * sig, 12 * sig, epsabs=0, epsrel=1e-13, limit=200)
        assert out[v[2], v[1], v[0]] == pytest.approx(ref, rel=1e-10)


def test_matrix_determinant_lemma_and_sherman_morrison():
    g = inputs.init_anisotropic(32, 50, np.random.default_rng(9))
    stk = inputs.stack_grid("sagittal", 32, 8, fwhm_slices=1.0)
    (gt, *_), = gauss.prepare(g, [stk])
    P = np.linalg.inv(gt["Sig_idx"])
    s2 = stk.psf_sigma_z ** 2
    amp_lemma = gt["wt"]["alpha"] / np.sqrt(1 + s2 * P[:, 2, 2])
    assert np.allclose(gt["amp"], amp_lemma, rtol=1e-12)
    pz = P[:, :, 2]
    C_sm = P - s2 * np.einsum("ni,nj->nij", pz, pz) / (1 + s2 * P[:, 2, 2])[:, None, None]
    assert np.allclose(gt["C"], C_sm, rtol=1e-9, atol=1e-12)


def test_box_contains_three_sigma_ellipsoid_and_is_tight():
    rng = np.random.default_rng(21)
    n = 28
    g = inputs.init_anisotropic(n, 200, rng)
    for grid in (inputs.volume_grid(n), inputs.stack_grid("axial", n, 7, 1.0),
                 inputs.stack_grid("coronal", n, 7, 1.0, *inputs.random_rigid(rng, 2, 1, n))):
        (gt, lo, hi, ne, valid), = gauss.prepare(g, [grid])
        assert valid.all()
        z, y, x = np.meshgrid(np.arange(grid.nz), np.arange(grid.ny), np.arange(grid.nx),
                              indexing="ij")
        v = np.stack([x, y, z], -1).reshape(-1, 3).astype(np.float64)
        for i in range(g.n):
            d = v - gt["c"][i]
            m2 = np.einsum("kj,jl,kl->k", d, gt["C"][i], d)
            inside = ((v >= lo[i]) & (v <= hi[i])).all(1)
            assert not np.any((m2 <= 9.0 - 1e-9) & ~inside)
            # tight: one voxel beyond the box along an axis is more than 3 sigma_j away
            sd = np.sqrt(np.diag(gt["Sig_g"][i]))
            for j in range(3):
                if lo[i, j] > 0:
                    assert gt["c"][i, j] - (lo[i, j] - 1) > 3 * sd[j] - 1e-9
                if hi[i, j] < grid.shape[::-1][j] - 1:
                    assert (hi[i, j] + 1) - gt["c"][i, j] > 3 * sd[j] - 1e-9


def test_box_width_for_sigma_1p1_at_voxel_centre_is_7():
    n = 32
    g = one([vox_world(15, n)] * 3, [1, 0, 0, 0], [math.log(1.1 * 2 / n)] * 3, [0])
    lo, hi, ne, _ = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, inputs.volume_grid(n))
    assert ne[0] and np.all(hi[0] - lo[0] + 1 == 7)


def test_box_recipe_vs_real_valued_boxes():
    """The recipe equals the real-valued 3-sigma box except possibly where a bound lies
    within rounding of an integer."""
    rng = np.random.default_rng(2)
    g = inputs.init_anisotropic(64, 3000, rng)
    grid = inputs.stack_grid("axial", 64, 16, 1.0)
    (gt, lo, hi, ne, _), = gauss.prepare(g, [grid])
    sd = np.sqrt(np.einsum("nii->ni", gt["Sig_g"]))
    lo_r = np.maximum(np.ceil(gt["c"] - 3 * sd), 0)
    hi_r = np.minimum(np.floor(gt["c"] + 3 * sd), np.array([63, 63, 15]))
    near = (np.abs((gt["c"] - 3 * sd) - np.rint(gt["c"] - 3 * sd)) < 1e-9) | \
           (np.abs((gt["c"] + 3 * sd) - np.rint(gt["c"] + 3 * sd)) < 1e-9)
    diff = ((lo_r != lo) | (hi_r != hi)) & ne[:, None]
    assert not np.any(diff & ~near)


def test_invalid_inputs_give_empty_boxes():
    g = inputs.init_anisotropic(16, 6, np.random.default_rng(1))
    g.quat[1] = 0
    g.mean[2, 0] = np.nan
    g.log_scale[3, 1] = np.inf
    g.logit[4] = np.nan
    g.log_scale[5, 2] = -1000.0
    lo, hi, ne, valid = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, inputs.volume_grid(16))
    assert valid.tolist() == [True, False, False, False, False, False]
    assert ne.tolist() == [True, False, False, False, False, False]


def test_box_outside_grid_is_empty_and_face_touching_is_clipped():
    n = 16
    g = one([1.8, 0.0, 0.0], [1, 0, 0, 0], [math.log(2 / n)] * 3, [0])
    lo, hi, ne, _ = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, inputs.volume_grid(n))
    assert not ne[0]
    g = one([1.0, -1.0, 0.0], [1, 0, 0, 0], [math.log(2 / n)] * 3, [0])
    lo, hi, ne, _ = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, inputs.volume_grid(n))
    assert ne[0] and hi[0, 0] == n - 1 and lo[0, 1] == 0


def test_c_brute_force_matches_numpy_and_permutation_invariance():
    rng = np.random.default_rng(4)
    n = 14
    g = inputs.init_anisotropic(n, 120, rng)
    g.log_scale += np.float32(0.4)
    grid = inputs.stack_grid("sagittal", n, 5, 1.0, *inputs.random_rigid(rng, 2, 1, n))
    (gt, lo, hi, ne, _), = gauss.prepare(g, [grid])
    a = gauss.render(grid, gt, lo, hi, ne)
    b = gauss.render_numpy(grid, gt, lo, hi, ne)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))
    perm = rng.permutation(g.n)
    (gt2, lo2, hi2, ne2, _), = gauss.prepare(g.subset(perm), [grid])
    c = gauss.render(grid, gt2, lo2, hi2, ne2)
    assert np.max(np.abs(a - c)) <= 1e-13 * np.max(np.abs(a))
    pts = np.array([[1, 2, 3], [5, 5, 1], [13, 0, 4]])
    p = gauss.render_points(pts, gt, lo, hi, ne)
    assert np.array_equal(p, a[pts[:, 2], pts[:, 1], pts[:, 0]])


def test_integer_shift_shifts_output():
    n = 20
    rng = np.random.default_rng(8)
    g = inputs.init_anisotropic(n, 40, rng)
    g.mean[:] = np.clip(g.mean, -0.5, 0.5)
    grid = inputs.volume_grid(n)
    shifted = g.mean.copy()
    shifted[:, 0] += np.float32(2 * 3 / n)
    h = inputs.Gaussians(shifted, g.quat, g.log_scale, g.logit)
    a = gauss.render_all(g, [grid])[0]
    b = gauss.render_all(h, [grid])[0]
    assert np.allclose(a[:, :, :-3], b[:, :, 3:], rtol=1e-5, atol=1e-9)


def test_tile_lists_against_brute_force_tile_enumeration():
    rng = np.random.default_rng(6)
    n = 23
    g = inputs.init_anisotropic(n, 150, rng)
    grid = inputs.stack_grid("axial", n, 9, 1.0)
    tile = (8, 4, 2)
    lo, hi, ne, _ = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, grid)
    tiles, gids = recipe.tile_lists(lo, hi, ne, grid, tile, base=5)
    T = recipe.n_tiles(grid, tile)
    ntx, nty = -(-n // 8), -(-n // 4)
    ref = []
    for t in range(T):
        tx, ty, tz = t % ntx, (t // ntx) % nty, t // (ntx * nty)
        t0 = np.array([tx * 8, ty * 4, tz * 2])
        t1 = np.minimum(t0 + np.array(tile) - 1, np.array([n - 1, n - 1, 8]))
        for i in range(g.n):
            if ne[i] and np.all(lo[i] <= t1) and np.all(hi[i] >= t0):
                ref.append((t + 5, i))
    assert list(zip(tiles.tolist(), gids.tolist())) == ref
    counts = recipe.tile_counts(lo, hi, ne, tile)
    assert counts.sum() == len(ref)


def test_devox_constant_stacks_partition_of_unity():
    """Constant stacks of value v: interior Gaussians get alpha = v 8/(2 pi)^{3/2}, and the
    rendered lattice of Gaussians reproduces v on average over whole lattice periods (Poisson
    summation: the lattice sum of sigma = h/2 Gaussians is (2 pi)^{3/2} sigma^3 / h^3 times
    1 + a ripple of period h whose mean over a period vanishes)."""
    n, g = 24, 8
    stacks = inputs.orthogonal_stacks(n, 6, 1.0)
    data = [np.full(s.shape, 0.7, np.float32) for s in stacks]
    mean, quat, ls, logit = gauss.devox_init(g, stacks, data)
    alpha = 1 / (1 + np.exp(-logit))
    inner = (np.abs(mean) < 0.7).all(1)
    assert np.allclose(alpha[inner], 0.7 * 8 / (2 * math.pi) ** 1.5, rtol=1e-12)
    gs = inputs.Gaussians(mean.astype(np.float32), quat.astype(np.float32),
                          ls.astype(np.float32), logit.astype(np.float32))
    vol = gauss.render_all(gs, [inputs.volume_grid(n)], cutoff=8.0)[0]
    core = vol[6:18, 6:18, 6:18]            # 12 voxels = 4 lattice periods (h = 3 voxels)
    assert core.mean() == pytest.approx(0.7, rel=2e-6)   # float32-stored alpha and sigma
    assert 0.02 < (core.max() - core.min()) / 0.7 < 0.1    # the ripple is there

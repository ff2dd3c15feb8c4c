"""Pins of the oracle's training iteration (oracle/train.py), its gradient-sensitivity sums and
its index->world recipe, against definitions that do not go through them."""
import numpy as np
import pytest

from oracle import gauss, recipe, train
from oracle import nrf as onrf
from paper_2603_00145_amd import inputs


def tiny(seed=0, n=12, ng=6):
    rng = np.random.default_rng(seed)
    g = inputs.init_anisotropic(n, ng, rng)
    grids = [inputs.stack_grid("axial", n, 4, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("sagittal", n, 3, 1.0)]
    targets = [rng.uniform(0, 1, size=gr.shape).astype(np.float32) for gr in grids]
    return g, grids, targets, rng


def test_index_to_world_is_the_inverse():
    rng = np.random.default_rng(3)
    for orient in ("axial", "coronal", "sagittal"):
        gr = inputs.stack_grid(orient, 40, 10, 1.0, *inputs.random_rigid(rng, 2, 1, 40))
        A = np.asarray(gr.world_to_index, np.float64)
        M = onrf.index_to_world(A)
        # M o A = identity on homogeneous points
        Ah = np.vstack([A, [0, 0, 0, 1]])
        Mh = np.vstack([M, [0, 0, 0, 1]])
        assert np.max(np.abs(Mh @ Ah - np.eye(4))) < 1e-14
        assert np.max(np.abs(M[:, :3] - np.linalg.inv(A[:, :3]))) < 1e-14 * np.abs(M).max()


def test_abs_jacobian_sums_brute_force():
    """Against a per-voxel complex step of each Gaussian rendered alone (render_numpy)."""
    g, grids, _, _ = tiny()
    got = gauss.abs_jacobian_sums(g, grids)
    sizes = (3, 4, 3, 1)
    for i in range(g.n):
        gi = g.subset([i])
        for grp, k in enumerate(sizes):
            for comp in range(k):
                tot = 0.0
                for gr in grids:
                    lo, hi, ne, _ = recipe.boxes(gi.mean, gi.quat, gi.log_scale, gi.logit, gr)
                    p = [np.asarray(a, np.complex128) for a in gauss.params64(gi)]
                    if p[grp].ndim == 1:
                        p[grp] = p[grp] + 1e-30j
                    else:
                        p[grp][:, comp] += 1e-30j
                    vals = gauss.render_numpy(gr, gauss.grid_terms(*p, gr), lo, hi, ne)
                    tot += np.abs(vals.imag / 1e-30).sum()
                ref = tot
                val = got[grp][i] if grp == 3 else got[grp][i, comp]
                assert abs(val - ref) <= 1e-12 * max(abs(ref), 1e-300)


def test_abs_jacobian_logit_is_the_unit_gradient():
    """d w / d logit = w (1 - alpha) > 0 at every voxel, so the absolute sum is the gradient of
    sum_v I[v] (dl = 1)."""
    g, grids, _, _ = tiny(seed=1)
    got = gauss.abs_jacobian_sums(g, grids)
    ref = gauss.gradients(g, grids, [np.ones(gr.shape) for gr in grids])
    assert np.max(np.abs(got[3] - ref[3])) <= 1e-12 * np.max(np.abs(ref[3]))
    # and bounds every other component of any gradient with |dl| <= 1
    rng = np.random.default_rng(2)
    dl = [rng.uniform(-1, 1, size=gr.shape) for gr in grids]
    anyg = gauss.gradients(g, grids, dl)
    for a, b in zip(anyg, got):
        assert np.all(np.abs(a) <= b * (1 + 1e-12) + 1e-300)


def loss_fp64(params, grids, targets, weights=None, field=None):
    """The data term from FP64 parameters, boxes from the float32 parameters (fixed)."""
    g32 = train._G(*[np.asarray(a, np.float32) for a in params])
    tot = 0.0
    ntot = sum(gr.n_voxels for gr in grids)
    for gr, y in zip(grids, targets):
        lo, hi, ne, _ = recipe.boxes(g32.mean, g32.quat, g32.log_scale, g32.logit, gr)
        gt = gauss.grid_terms(*[np.asarray(a, np.float64) for a in params], gr)
        I = gauss.render_numpy(gr, gt, lo, hi, ne)
        if weights is not None:
            x = onrf.world_coords(train.all_voxels(gr), onrf.index_to_world(gr.world_to_index))
            r, *_ = onrf.forward(weights, onrf.encode(x, field["n_freq"], field["in_pad"]),
                                 field["out_scale"])
            I = I + r.reshape(gr.shape)
        d = I - np.asarray(y, np.float64)
        ad = np.abs(d)
        tot += np.where(ad < 1, 0.5 * d * d, ad - 0.5).sum()
    return tot / ntot


def test_step_gradients_central_differences():
    """The step's raw gradients (data term + anisotropy) against central differences of the
    loss written out in FP64 (boxes fixed), and its Adam step's first-step closed form."""
    g, grids, targets, rng = tiny(seed=4)
    params = [g.mean, g.quat, g.log_scale, g.logit]
    z = [np.zeros(np.shape(a)) for a in params]
    lam_a, lam_r = 0.1, 1.2
    lrs = (1e-3, 1e-3, 5e-3, 5e-2)
    out = train.step(params, z, z, 1, grids, targets, lrs, lam_a, lam_r)
    assert out["loss"] == pytest.approx(loss_fp64(params, grids, targets), rel=1e-13)
    p64 = [np.asarray(a, np.float32).astype(np.float64) for a in params]
    for grp, k in enumerate((3, 4, 3, 1)):
        for i in range(g.n):
            for comp in range(k):
                h = 1e-6
                vals = []
                for s in (1, -1):
                    pp = [a.copy() for a in p64]
                    if grp == 3:
                        pp[3][i] += s * h
                    else:
                        pp[grp][i, comp] += s * h
                    L = loss_fp64(pp, grids, targets)
                    # Eq. 13 on the actual scales, mean over the Gaussians, in FP64
                    D = pp[2].max(1) - pp[2].min(1)
                    L += lam_a * np.maximum(np.exp(D) - lam_r, 0.0).mean()
                    vals.append(L)
                fd = (vals[0] - vals[1]) / (2 * h)
                an = out["grads"][grp][i] if grp == 3 else out["grads"][grp][i, comp]
                scale = np.max(np.abs(out["grads"][grp]))
                assert abs(an - fd) <= 1e-6 * scale + 1e-12
        # Adam's first step: p - lr g / (|g| + eps)
        gr = out["grads"][grp]
        ref = p64[grp] - lrs[grp] * gr / (np.abs(gr) + 1e-8)
        assert np.max(np.abs(out["p"][grp] - ref)) <= 1e-15


def test_step_field_gradient_central_differences():
    """With the residual field on: the loss includes r at every stack voxel, and the field's
    weight gradients match central differences of the FP64 loss in the weights."""
    g, grids, targets, rng = tiny(seed=5, n=10, ng=4)
    params = [g.mean, g.quat, g.log_scale, g.logit]
    z = [np.zeros(np.shape(a)) for a in params]
    depth, n_freq, in_pad = 2, 4, 64
    master = {"w_in": rng.uniform(-0.3, 0.3, (64, in_pad)).astype(np.float32),
              "b_in": rng.uniform(-0.1, 0.1, 64).astype(np.float32),
              "w_hid": rng.uniform(-0.2, 0.2, (1, 64, 64)).astype(np.float32),
              "b_hid": rng.uniform(-0.1, 0.1, (1, 64)).astype(np.float32),
              "w_out": rng.uniform(-0.2, 0.2, 64).astype(np.float32),
              "b_out": np.array([0.05], np.float32)}
    master["w_in"][:, 3 + 6 * n_freq:] = 0
    zz = {k: np.zeros(v.shape) for k, v in master.items()}
    field = dict(master=master, m=zz, v=zz, t=1, lr=1e-4, n_freq=n_freq, in_pad=in_pad,
                 depth=depth, out_scale=0.1)
    out = train.step(params, z, z, 1, grids, targets, (1e-3,) * 4, 0.0, 1.5, field)
    W = train.field_weights(master, depth)
    assert out["loss"] == pytest.approx(loss_fp64(params, grids, targets, W, field), rel=1e-13)
    checks = [("w_out", lambda w: w["w_out"], (5,)), ("b_out", None, ()),
              ("w_in", lambda w: w["W"][0], (7, 2)), ("w_hid", lambda w: w["W"][1], (3, 11)),
              ("b_in", lambda w: w["b"][0], (9,)), ("b_hid", lambda w: w["b"][1], (13,))]
    fg = out["field_grads"]
    for name, get, ix in checks:
        h = 1e-6
        vals = []
        for s in (1, -1):
            w2 = {"W": [a.copy() for a in W["W"]], "b": [a.copy() for a in W["b"]],
                  "w_out": W["w_out"].copy(), "b_out": W["b_out"]}
            if name == "b_out":
                w2["b_out"] += s * h
            else:
                get(w2)[ix] += s * h
            vals.append(loss_fp64(params, grids, targets, w2, field))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = fg["b_out"].reshape(-1)[0] if name == "b_out" else \
            (fg[name][0][ix] if name in ("w_hid", "b_hid") else fg[name][ix])
        assert abs(an - fd) <= 1e-6 * max(np.max(np.abs(fg[name])), 1e-12), name


def test_scatter_render_equals_brute_force():
    """Each Gaussian visiting its own box gives the brute-force sums bit for bit (same terms,
    same ascending order per voxel), on rotated stacks and a volume."""
    rng = np.random.default_rng(8)
    n = 23
    g = inputs.init_anisotropic(n, 400, rng)
    grids = [inputs.stack_grid("coronal", n, 6, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.volume_grid(n)]
    for gr, (gt, lo, hi, ne, _) in zip(grids, gauss.prepare(g, grids)):
        a = gauss.render(gr, gt, lo, hi, ne)
        b = gauss.render_scatter(gr, gt, lo, hi, ne)
        assert np.array_equal(a, b)

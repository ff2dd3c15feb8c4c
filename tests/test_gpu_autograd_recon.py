"""Autograd wrapper, gradcheck against FP64 central differences, devoxelization init and
reconstruction convergence."""
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


def normwise(gpu, ref):
    ref = np.asarray(ref, np.float64)
    s = np.max(np.abs(ref)) if ref.size else 0.0
    d = np.max(np.abs(np.asarray(gpu, np.float64) - ref)) if ref.size else 0.0
    return d / s if s > 0 else d


@pytest.fixture(scope="module")
def mods():
    from paper_2603_00145_amd import api, autograd
    api.load()
    return api, autograd


def crop_subset(w, lo_vox, size):
    """The Gaussians whose centres fall in the crop [lo_vox, lo_vox + size)^3 of the volume."""
    idx = (w.gauss.mean.astype(np.float64) + 1) * w.n_vox / 2 - 0.5
    inside = np.all((idx >= lo_vox - 0.5) & (idx < lo_vox + size - 0.5), axis=1)
    return w.gauss.subset(np.nonzero(inside)[0])


def single_gaussian_loss(params, grid, dl, lo, hi):
    """sum over one Gaussian's box of dl * its value (FP64 parameters, numpy), box fixed."""
    mean, quat, ls, logit = params
    gt = gauss.grid_terms(mean, quat, ls, logit, grid)
    z, y, x = np.meshgrid(np.arange(lo[2], hi[2] + 1), np.arange(lo[1], hi[1] + 1),
                          np.arange(lo[0], hi[0] + 1), indexing="ij")
    v = np.stack([x, y, z], -1).reshape(-1, 3).astype(np.float64)
    d = v - gt["c"][0]
    q = np.einsum("kj,jl,kl->k", d, gt["C"][0], d)
    w = gt["amp"][0] * np.exp(-0.5 * q)
    return float((w * dl[z, y, x].reshape(-1)).sum())


def test_gradcheck_c256_crop_subset(mods):
    """The ~1k Gaussians of a 26^3 crop of the 256^3 workload, rendered onto the three full
    256x256x64 stacks through the autograd Function; gradients against the oracle's analytic
    FP64 gradients (all components) and FP64 central differences (sampled components)."""
    api, autograd = mods
    w = inputs.workload("c256", with_data=False)
    g = crop_subset(w, 115, 26)
    say("gradcheck subset size", g.n)
    assert 800 <= g.n <= 1400
    rng = np.random.default_rng(5)
    dl = inputs.random_dl_di(w.stacks, rng)
    p = [torch.from_numpy(np.ascontiguousarray(getattr(g, k))).cuda().requires_grad_(True)
         for k in ("mean", "quat", "log_scale", "logit")]
    b = api.Bins(g.n, w.stacks)
    outs = autograd.render(p, b, [0, 1, 2])
    L = sum((o * torch.from_numpy(d).cuda()).sum() for o, d in zip(outs, dl))
    L.backward()
    got = [t.grad.cpu().numpy() for t in p]
    ref = gauss.gradients(g, w.stacks, dl)
    for name, a, r in zip(("mean", "quat", "log_scale", "logit"), got, ref):
        err = normwise(a, r)
        say(f"  autograd vs oracle {name}: {err:.2e}")
        assert err <= TOL
    # FP64 central differences on sampled components (boxes held fixed)
    boxes = [recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, s)[:3] for s in w.stacks]
    fd, an, gpu = [], [], []
    for trial in range(40):
        i = int(rng.integers(g.n))
        k = int(rng.integers(4))
        comp = int(rng.integers([3, 4, 3, 1][k]))
        base = [np.asarray(getattr(g.subset([i]), f), np.float32).astype(np.float64)
                for f in ("mean", "quat", "log_scale", "logit")]
        theta = base[k].reshape(-1)[comp]
        h = 1e-6 * max(1.0, abs(theta))
        vals = []
        for sgn in (1, -1):
            pert = [x.copy() for x in base]
            pert[k].reshape(-1)[comp] += sgn * h
            tot = 0.0
            for s, d, (lo, hi, ne) in zip(w.stacks, dl, boxes):
                if ne[i]:
                    tot += single_gaussian_loss(pert, s, d, lo[i], hi[i])
            vals.append(tot)
        fd.append((vals[0] - vals[1]) / (2 * h))
        an.append(ref[k].reshape(g.n, -1)[i, comp])
        gpu.append(got[k].reshape(g.n, -1)[i, comp])
    fd, an, gpu = map(np.array, (fd, an, gpu))
    say(f"  oracle analytic vs FD: {normwise(an, fd):.2e}; GPU vs FD: {normwise(gpu, fd):.2e}")
    assert normwise(an, fd) <= 1e-6
    assert normwise(gpu, fd) <= TOL


def test_two_forwards_before_backward(mods):
    """Two forwards on the same bins (the second with other parameters re-bins them) before
    the first forward's backward: the first backward still differentiates its own parameters."""
    api, autograd = mods
    rng = np.random.default_rng(31)
    n = 30
    g1 = inputs.init_anisotropic(n, 400, rng)
    g2 = inputs.init_anisotropic(n, 400, rng)
    grids = [inputs.stack_grid("axial", n, 8, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.volume_grid(n)]
    dl = inputs.random_dl_di(grids, rng)
    b = api.Bins(g1.n, grids)

    def leaf(g):
        return [torch.from_numpy(np.ascontiguousarray(getattr(g, k))).cuda().requires_grad_(True)
                for k in ("mean", "quat", "log_scale", "logit")]

    p1, p2 = leaf(g1), leaf(g2)
    o1 = autograd.render(p1, b, [0, 1])
    o2 = autograd.render(p2, b, [0, 1])          # re-bins b for g2
    L1 = sum((o * torch.from_numpy(d).cuda()).sum() for o, d in zip(o1, dl))
    L2 = sum((o * torch.from_numpy(d).cuda()).sum() for o, d in zip(o2, dl))
    L1.backward()
    L2.backward()
    for g, p in ((g1, p1), (g2, p2)):
        ref = gauss.gradients(g, grids, dl)
        for name, t, r in zip(("mean", "quat", "log_scale", "logit"), p, ref):
            err = normwise(t.grad.cpu().numpy(), r)
            assert err <= TOL, (name, err)


def test_devox_matches_oracle(mods):
    api, _ = mods
    w = inputs.workload("c64")
    data = [torch.from_numpy(d).cuda() for d in w.stack_data]
    for G in (1, 7, 16):
        p = api.devox_init(G, w.stacks, data)
        torch.cuda.synchronize()
        mean, quat, ls, logit = gauss.devox_init(G, w.stacks, w.stack_data)
        assert np.allclose(p.mean.cpu().numpy(), mean, rtol=0, atol=1e-6)
        assert np.array_equal(p.quat.cpu().numpy(), quat.astype(np.float32))
        assert np.allclose(p.log_scale.cpu().numpy(), ls, rtol=1e-6)
        a_gpu = 1 / (1 + np.exp(-p.logit.cpu().numpy().astype(np.float64)))
        a_ref = 1 / (1 + np.exp(-logit))
        assert normwise(a_gpu, a_ref) <= TOL


def test_reconstruction_converges_c64(mods):
    api, _ = mods
    from paper_2603_00145_amd import recon
    w = inputs.workload("c64", device="cuda")
    g = inputs.init_anisotropic(64, 20000, np.random.default_rng(0))
    p = api.GaussParams.from_host(g)
    r = recon.Reconstruction(w.stacks, w.stack_data, p, recon.TrainConfig(n_iter=150),
                             w.volume, w.phantom)
    hist = r.run()
    say("  c64 psnr", [round(h["psnr"], 2) for h in hist[::3]])
    losses = [h["loss"] for h in hist if h["loss"] is not None]
    assert losses[-1] < 0.5 * losses[0]
    assert hist[-1]["psnr"] > hist[0]["psnr"] + 3.0

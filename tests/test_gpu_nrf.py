"""Neural residual field on MFMA (BF16 weights/activations, FP32 accumulation) against the
FP64 oracle with the same BF16-valued weights: bar 2e-2 normwise per output."""
import sys

import numpy as np
import pytest
import torch

from oracle import nrf as onrf
from precision_report import row as report
from paper_2603_00145_amd import inputs

pytestmark = pytest.mark.gpu
TOL_BF16 = 2e-2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(gpu, ref):
    ref = np.asarray(ref, np.float64)
    return np.max(np.abs(np.asarray(gpu, np.float64) - ref)) / max(np.max(np.abs(ref)), 1e-30)


@pytest.fixture(scope="module")
def mods():
    from paper_2603_00145_amd import _lib, api, nrf
    api.load()
    return _lib, api, nrf


def all_voxels(grid):
    z, y, x = np.meshgrid(np.arange(grid.nz), np.arange(grid.ny), np.arange(grid.nx), indexing="ij")
    return np.stack([x, y, z], -1).reshape(-1, 3)


@pytest.mark.parametrize("n_freq,depth", [(16, 3), (6, 4)])
def test_nrf_forward_parity(mods, n_freq, depth):
    _lib, api, nrf = mods
    rng = np.random.default_rng(n_freq)
    grid = inputs.stack_grid("coronal", 33, 9, 1.0, *inputs.random_rigid(rng, 2, 1, 33))
    net = nrf.NRF(n_freq=n_freq, depth=depth, seed=3, zero_last=False)
    base = torch.from_numpy(rng.normal(size=grid.shape).astype(np.float32)).cuda()
    out = base.clone()
    net.forward_add(grid, out)
    torch.cuda.synchronize()
    r_gpu = (out - base).cpu().numpy().reshape(-1)
    x = onrf.world_coords(all_voxels(grid), onrf.index_to_world(grid.world_to_index))
    r_ref, *_ = onrf.forward(net.weights_host(), onrf.encode(x, n_freq, net.in_pad), net.out_scale)
    err = normwise(r_gpu, r_ref)
    report(f"33x33x9 stack, L={n_freq} D={depth}", "field r, every voxel", "BF16 MFMA, FP32 acc.",
           r_gpu, r_ref)
    say(f"  nrf forward L={n_freq} D={depth}: normwise {err:.2e}, max|r| {np.abs(r_ref).max():.3f}")
    assert err <= TOL_BF16


@pytest.mark.parametrize("n_freq,depth", [(16, 3), (6, 4)])
def test_nrf_backward_parity(mods, n_freq, depth):
    _lib, api, nrf = mods
    rng = np.random.default_rng(7 + depth)
    grid = inputs.stack_grid("axial", 40, 10, 1.0, *inputs.random_rigid(rng, 2, 1, 40))
    net = nrf.NRF(n_freq=n_freq, depth=depth, seed=5, zero_last=False)
    dl = rng.normal(size=grid.shape).astype(np.float32)
    idx = rng.choice(grid.n_voxels, size=3001, replace=False).astype(np.int32)
    net.zero_grad()
    _, scale = net.backward(grid, torch.from_numpy(dl).cuda(), idx=torch.from_numpy(idx).cuda())
    torch.cuda.synchronize()
    vox = all_voxels(grid)[idx]
    x = onrf.world_coords(vox, onrf.index_to_world(grid.world_to_index))
    feats = onrf.encode(x, n_freq, net.in_pad)
    g = onrf.backward(net.weights_host(), feats, dl.reshape(-1)[idx].astype(np.float64) * scale,
                      net.out_scale)
    got = {k: v.cpu().numpy() for k, v in net.g.items()}
    checks = [("w_in", got["w_in"], g["W"][0]), ("b_in", got["b_in"], g["b"][0]),
              ("w_out", got["w_out"], g["w_out"]), ("b_out", got["b_out"][0], g["b_out"])]
    for l in range(depth - 1):
        checks += [(f"w_hid{l}", got["w_hid"][l], g["W"][l + 1]), (f"b_hid{l}", got["b_hid"][l], g["b"][l + 1])]
    for name, a, r in checks:
        err = normwise(a, r)
        say(f"  nrf backward L={n_freq} D={depth} {name}: {err:.2e}")
        assert err <= TOL_BF16, name


def test_nrf_backward_parity_training_size(mods):
    """The field's gradient as training takes it on the 256^3 workload: 2^18 sampled voxels of
    a rigidly offset 256x256x64 stack, 16 bands, three 64-wide layers (the split-K weight
    gradients then sum 256 partials per element)."""
    _lib, api, nrf = mods
    rng = np.random.default_rng(12)
    grid = inputs.stack_grid("coronal", 256, 64, 1.0, *inputs.random_rigid(rng, 2, 1, 256))
    net = nrf.NRF(n_freq=16, depth=3, seed=9, zero_last=False)
    dl = (rng.normal(size=grid.shape) * 1e-6).astype(np.float32)
    npts = 1 << 18
    idx = rng.choice(grid.n_voxels, size=npts, replace=False).astype(np.int32)
    net.zero_grad()
    _, scale = net.backward(grid, torch.from_numpy(dl).cuda(), idx=torch.from_numpy(idx).cuda())
    torch.cuda.synchronize()
    assert scale == grid.n_voxels / npts
    z, rem = np.divmod(idx.astype(np.int64), grid.nx * grid.ny)
    y, x = np.divmod(rem, grid.nx)
    vox = np.stack([x, y, z], 1)
    xw = onrf.world_coords(vox, onrf.index_to_world(grid.world_to_index))
    feats = onrf.encode(xw, 16, net.in_pad)
    g = onrf.backward(net.weights_host(), feats, dl.reshape(-1)[idx].astype(np.float64) * scale,
                      net.out_scale)
    got = {k: v.cpu().numpy() for k, v in net.g.items()}
    checks = [("w_in", got["w_in"], g["W"][0]), ("b_in", got["b_in"], g["b"][0]),
              ("w_out", got["w_out"], g["w_out"]), ("b_out", got["b_out"][0], g["b_out"])]
    for l in range(2):
        checks += [(f"w_hid{l}", got["w_hid"][l], g["W"][l + 1]),
                   (f"b_hid{l}", got["b_hid"][l], g["b"][l + 1])]
    for name, a, r in checks:
        err = normwise(a, r)
        report("256x256x64 stack, 2^18 sampled voxels", f"field dL/d{name}",
               "BF16 MFMA, FP32 acc.", a, r)
        say(f"  nrf backward 2^18 points {name}: {err:.2e}")
        assert err <= TOL_BF16, name


def test_nrf_backward_over_several_grids(mods):
    """One backward call over three grids (3001 and 17 sampled voxels, and every voxel of a
    third grid): the oracle's gradient summed over the grids, and the three single-grid calls
    up to the order of the FP32 sums.  Every gradient is a sum over points of per-point terms
    that BF16 storage perturbs by a few units of 2^-8 each; with random-sign dl_dr a bias sum
    can cancel far below its terms, so the oracle bar is taken relative to the sum of the
    terms' magnitudes (the oracle's gradient at each point alone), the usual bound of a
    rounded sum."""
    _lib, api, nrf = mods
    rng = np.random.default_rng(21)
    grids = [inputs.stack_grid("axial", 40, 10, 1.0, *inputs.random_rigid(rng, 2, 1, 40)),
             inputs.stack_grid("coronal", 24, 6, 1.0, *inputs.random_rigid(rng, 2, 1, 24)),
             inputs.stack_grid("sagittal", 20, 3, 1.5, *inputs.random_rigid(rng, 2, 1, 20))]
    net = nrf.NRF(n_freq=16, depth=3, seed=6, zero_last=False)
    dls = [rng.normal(size=g.shape).astype(np.float32) for g in grids]
    idxs = [rng.choice(grids[0].n_voxels, size=3001, replace=False).astype(np.int32),
            rng.choice(grids[1].n_voxels, size=17, replace=False).astype(np.int32), None]
    dls_d = [torch.from_numpy(d).cuda() for d in dls]
    idx_d = [None if i is None else torch.from_numpy(i).cuda() for i in idxs]
    net.zero_grad()
    say("  nrf backward over 3 grids: one call")
    _, scales = net.backward_grids(grids, dls_d, idxs=idx_d)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in net.g.items()}
    # a fourth grid with an empty sample changes nothing
    net.zero_grad()
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    net.backward_grids(grids + [grids[0]], dls_d + [dls_d[0]], idxs=idx_d + [empty])
    torch.cuda.synchronize()
    for k, v in net.g.items():
        assert normwise(v.cpu().numpy(), got[k]) <= 1e-5, f"{k} with an empty grid"
    net.zero_grad()
    for g, d, i in zip(grids, dls_d, idx_d):
        net.backward(g, d, idx=i)
    torch.cuda.synchronize()
    one = {k: v.cpu().numpy().astype(np.float64) for k, v in net.g.items()}
    def flat(g):
        return {"w_in": g["W"][0], "b_in": g["b"][0], "w_out": g["w_out"], "b_out": g["b_out"],
                "w_hid0": g["W"][1], "b_hid0": g["b"][1], "w_hid1": g["W"][2], "b_hid1": g["b"][2]}

    wts = net.weights_host()
    ref, mag = {}, {}
    for g, d, i, sc in zip(grids, dls, idxs, scales):
        vox = all_voxels(g) if i is None else all_voxels(g)[i]
        x = onrf.world_coords(vox, onrf.index_to_world(g.world_to_index))
        dsel = (d.reshape(-1) if i is None else d.reshape(-1)[i]).astype(np.float64) * sc
        feats = onrf.encode(x, 16, net.in_pad)
        for k, v in flat(onrf.backward(wts, feats, dsel, net.out_scale)).items():
            ref[k] = ref.get(k, 0.0) + np.asarray(v)
        for p in range(len(dsel)):
            for k, v in flat(onrf.backward(wts, feats[p:p + 1], dsel[p:p + 1], net.out_scale)).items():
                mag[k] = mag.get(k, 0.0) + np.abs(np.asarray(v))
    where = {"w_in": ("w_in", None), "b_in": ("b_in", None), "w_out": ("w_out", None),
             "b_out": ("b_out", 0), "w_hid0": ("w_hid", 0), "b_hid0": ("b_hid", 0),
             "w_hid1": ("w_hid", 1), "b_hid1": ("b_hid", 1)}
    for name, (key, sel) in where.items():
        a = got[key] if sel is None else got[key][sel]
        b = one[key] if sel is None else one[key][sel]
        e_ref = np.max(np.abs(a - ref[name])) / np.max(mag[name])
        e_one = normwise(a, b)
        say(f"  nrf backward 3 grids {name}: oracle {e_ref:.2e} (of the terms' magnitudes), "
            f"normwise {normwise(a, ref[name]):.2e}; single-grid calls {e_one:.2e}")
        assert e_ref <= TOL_BF16, name
        assert e_one <= 1e-5, name


def test_nrf_backward_over_several_grids_training_size(mods):
    """The one-call backward as training takes it (2^18 sampled voxels on each of three
    256x256x64 stacks) against the three single-grid calls: the same dZ and activations, only
    the split of the weight-gradient sums over the points differs (to 1e-5)."""
    _lib, api, nrf = mods
    w = inputs.workload("c256", with_data=False)
    rng = np.random.default_rng(31)
    net = nrf.NRF(n_freq=16, depth=3, seed=4, zero_last=False)
    dls = [torch.from_numpy((rng.normal(size=g.shape) * 1e-6).astype(np.float32)).cuda()
           for g in w.stacks]
    idxs = [torch.from_numpy(rng.choice(g.n_voxels, size=1 << 18, replace=False)
                             .astype(np.int32)).cuda() for g in w.stacks]
    say("  nrf backward, 3 x 2^18 points: one call against three")
    net.zero_grad()
    net.backward_grids(w.stacks, dls, idxs=idxs)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in net.g.items()}
    net.zero_grad()
    for g, d, i in zip(w.stacks, dls, idxs):
        net.backward(g, d, idx=i)
    torch.cuda.synchronize()
    for k, v in net.g.items():
        err = normwise(got[k], v.cpu().numpy())
        say(f"  {k}: {err:.2e}")
        assert err <= 1e-5, k


def test_render_volume_with_nrf(mods):
    _lib, api, nrf = mods
    g = inputs.init_anisotropic(20, 200, np.random.default_rng(1))
    vol = inputs.volume_grid(20)
    p = api.GaussParams.from_host(g)
    b = api.Bins(p.n, [vol])
    b.bin(p)
    net = nrf.NRF(n_freq=8, depth=3, seed=2, zero_last=False)
    plain = api.render_volume(b, 0)
    with_r = api.render_volume(b, 0, nrf=net)
    extra = plain.clone()
    net.forward_add(vol, extra)
    torch.cuda.synchronize()
    assert torch.equal(with_r, extra)
    assert float((with_r - plain).abs().max()) > 1e-4


@pytest.mark.parametrize("n_freq,depth", [(16, 3), (6, 2)])
def test_fused_render_field_loss(mods, n_freq, depth):
    """gm_render_nrf_loss_smooth_l1 (render + field + smooth-L1 in one pass) against the three
    calls it fuses, on ragged rotated stacks and a ragged volume: renderings and dL/dI bit for
    bit, the loss to 1e-6 (the order of its FP64 sum differs)."""
    _lib, api, nrf = mods
    rng = np.random.default_rng(7 + depth)
    n = 41
    g = inputs.init_anisotropic(n, 900, rng)
    grids = [inputs.stack_grid("axial", n, 11, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("coronal", n, 9, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("sagittal", n, 13, 1.0),
             inputs.volume_grid(n)]
    ids = [0, 1, 2, 3]
    say(f"fused render + field + loss: n_freq {n_freq} depth {depth}")
    targ = [torch.from_numpy(rng.normal(0.3, 1.0, size=gr.shape).astype(np.float32)).cuda()
            for gr in grids]
    b = api.Bins(g.n, grids)
    b.bin(api.GaussParams.from_host(g))
    net = nrf.NRF(n_freq=n_freq, depth=depth, seed=3, zero_last=False)
    outs = api.render(b, ids)
    for k in ids:
        net.forward_add(grids[k], outs[k])
    ref_loss, ref_dl = api.smooth_l1(outs, targ)
    stored = [torch.full(gr.shape, float("nan"), device="cuda") for gr in grids]
    loss, dl = api.render_loss(b, ids, targ, outs=stored, nrf=net)
    loss2, dl2 = api.render_loss(b, ids, targ, nrf=net)
    vol = api.render_volume(b, 3, nrf=net)
    torch.cuda.synchronize()
    for k in ids:
        assert torch.equal(stored[k], outs[k]), f"grid {k}: rendering + field differs"
        assert torch.equal(dl[k], ref_dl[k]), f"grid {k}: dL/dI differs"
        assert torch.equal(dl2[k], dl[k])
    assert torch.equal(vol, outs[3])
    assert float(loss2) == float(loss)
    assert float(loss) == pytest.approx(float(ref_loss), rel=1e-6)
    plain = api.render(b, ids)
    assert max(float((o - q).abs().max()) for o, q in zip(outs, plain)) > 1e-4  # field is on


def test_reconstruction_with_nrf_runs(mods):
    _lib, api, nrf = mods
    from paper_2603_00145_amd import recon
    w = inputs.workload("c64", device="cuda")
    g = inputs.init_anisotropic(64, 20000, np.random.default_rng(0))
    net = nrf.NRF(n_freq=16, depth=3, seed=0)
    cfg = recon.TrainConfig(n_iter=80, nrf=net, nrf_start=0.5, lr_nrf=1e-3)
    r = recon.Reconstruction(w.stacks, w.stack_data, api.GaussParams.from_host(g), cfg, w.volume,
                             w.phantom)
    hist = r.run()
    say("  psnr with nrf", [round(h["psnr"], 2) for h in hist])
    assert r.nrf_on
    assert float(net.p["w_out"].abs().max()) > 0          # the field has started learning
    assert hist[-1]["psnr"] > hist[0]["psnr"]

"""Neural residual field on MFMA (BF16 weights/activations, FP32 accumulation) against the
FP64 oracle with the same BF16-valued weights: bar 2e-2 normwise per output."""
import sys

import numpy as np
import pytest
import torch

from oracle import nrf as onrf
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
        say(f"  nrf backward 2^18 points {name}: {err:.2e}")
        assert err <= TOL_BF16, name


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

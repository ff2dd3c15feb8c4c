"""Full-size parity at the three larger workloads (128^3 with rigid offsets and bias, the
256^3 benchmark configuration, 320^3 with two oblique stacks and overlapping thick slices),
on sampled outputs the oracle computes one by one; and the 320^3 volume with the neural
residual field: FP32 (Gaussians) and BF16 (field) errors against FP64 on a 64^3 crop."""
import sys

import numpy as np
import pytest
import torch

from adam_bounds import adam_range, check_range
from precision_report import row as report
from oracle import gauss, recipe
from oracle import nrf as onrf
from paper_2603_00145_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-5
TOL_BF16 = 2e-2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(gpu, ref):
    ref = np.asarray(ref, np.float64)
    s = np.max(np.abs(ref)) if ref.size else 0.0
    d = np.max(np.abs(np.asarray(gpu, np.float64) - ref)) if ref.size else 0.0
    return d / s if s > 0 else d


def elementwise(gpu, ref):
    """Largest per-element relative error over the elements with |ref| >= 1e-3 max|ref|."""
    ref = np.asarray(ref, np.float64)
    big = np.abs(ref) >= 1e-3 * np.max(np.abs(ref))
    return float(np.max(np.abs(np.asarray(gpu, np.float64)[big] - ref[big]) / np.abs(ref[big])))


@pytest.fixture(scope="module")
def mods():
    from paper_2603_00145_amd import _lib, api, nrf
    api.load()
    return _lib, api, nrf


@pytest.mark.parametrize("name", ["c128", "c256", "c320"])
def test_full_size_sampled_parity(mods, name):
    """Every Gaussian on every stack: boxes, tile counts and pair totals bit-exact; tile lists
    bit-exact on sampled tiles; voxel values at sampled voxels and the gradients of sampled
    Gaussians (with the anisotropy term) against the oracle."""
    _lib, api, _ = mods
    w = inputs.workload(name, with_data=False)
    say(f"{name}: {w.gauss.n} Gaussians, {len(w.stacks)} stacks")
    rng = np.random.default_rng(9)
    p = api.GaussParams.from_host(w.gauss)
    G = len(w.stacks)
    ids = list(range(G))
    b = api.Bins(p.n, w.stacks, capacity=int(12 * p.n * G))
    b.bin(p)
    outs = api.render(b, ids)
    dl = inputs.random_dl_di(w.stacks, rng)
    grads = api.GaussParams.zeros_like(p)
    api.backward(p, b, ids, [torch.from_numpy(d).cuda() for d in dl], grads, 0.1, 1.5)
    torch.cuda.synchronize()
    tile = _lib.tile_dims()
    ts = b.tile_start.cpu().numpy()
    pg = (b.pair_gauss[:b.n_pairs].cpu().numpy().view(np.uint32) & 0x7FFFFFFF).astype(np.int64)
    prep = gauss.prepare(w.gauss, w.stacks)
    for k, (grid, (gt, lo, hi, ne, _)) in enumerate(zip(w.stacks, prep)):
        glo, ghi = (t.cpu().numpy() for t in b.boxes(k))
        assert np.array_equal((glo <= ghi).all(1), ne)
        assert np.array_equal(glo[ne], lo[ne]) and np.array_equal(ghi[ne], hi[ne])
        assert np.array_equal(b.tile_count[k].cpu().numpy(), recipe.tile_counts(lo, hi, ne, tile))
        assert b.pair_count(k) == int(recipe.box_volume(lo, hi, ne).sum())
        T = np.asarray(tile)
        ntx, nty = -(-grid.nx // T[0]), -(-grid.ny // T[1])
        for t in rng.integers(0, recipe.n_tiles(grid, tile), size=40):
            tx, ty, tz = t % ntx, (t // ntx) % nty, t // (ntx * nty)
            t0 = np.array([tx, ty, tz]) * T
            t1 = t0 + T - 1
            ref = np.nonzero(ne & np.all(lo <= t1, 1) & np.all(hi >= t0, 1))[0]
            gt_id = b.tile_base_host[k] + t
            assert np.array_equal(pg[ts[gt_id]:ts[gt_id + 1]], ref)
        pts = np.stack([rng.integers(0, grid.nx, 600), rng.integers(0, grid.ny, 600),
                        rng.integers(0, grid.nz, 600)], 1)
        ref = gauss.render_points(pts, gt, lo, hi, ne)
        got = outs[k].cpu().numpy()[pts[:, 2], pts[:, 1], pts[:, 0]]
        err = normwise(got, ref)
        report(name, f"stack {k} ({grid.name}) I, 600 sampled voxels", "FP32", got, ref)
        say(f"  {name} grid {k} ({grid.name}): {b.pair_count(k)} pairs, sampled voxel error {err:.2e}")
        assert err <= TOL
    sub = np.sort(rng.choice(p.n, 3000, replace=False))
    mean, quat, ls, logit = gauss.params64(w.gauss.subset(sub))
    parts = []
    for grid, (gt, lo, hi, ne, _), d in zip(w.stacks, prep, dl):
        gs = {"c": gt["c"][sub], "C": gt["C"][sub], "amp": gt["amp"][sub]}
        parts.append(gauss.grid_partials(grid, gs, lo[sub], hi[sub], ne[sub], d))
    ref = list(gauss.chain(mean, quat, ls, logit, w.stacks, parts))
    ref[2] = ref[2] + 0.1 * gauss.aniso(w.gauss.log_scale, 1.5)[1][sub]
    for pname, t, r in zip(("mean", "quat", "log_scale", "logit"), grads.tensors(), ref):
        err = normwise(t.cpu().numpy()[sub], r)
        report(name, f"dL/d{pname}, 3000 sampled Gaussians (random dL/dI)", "FP32",
               t.cpu().numpy()[sub], r)
        say(f"  {name} sampled gradient {pname}: {err:.2e}")
        assert err <= TOL


def test_c320_volume_crop_fp32_and_bf16(mods):
    """The 320^3 volume rendered from 2M Gaussians, with and without a BF16 neural residual
    field (16 frequency bands, three 64-wide layers), on the crop [128, 192)^3."""
    _lib, api, nrf = mods
    w = inputs.workload("c320", with_data=False)
    p = api.GaussParams.from_host(w.gauss)
    vb = api.Bins(p.n, [w.volume])
    vb.bin(p)
    plain = api.render_volume(vb, 0)
    net = nrf.NRF(n_freq=16, depth=3, seed=11, zero_last=False)
    full = api.render_volume(vb, 0, nrf=net)
    torch.cuda.synchronize()
    c0, size = 128, 64
    sl = slice(c0, c0 + size)
    g_plain = plain[sl, sl, sl].cpu().numpy().reshape(-1)
    g_full = full[sl, sl, sl].cpu().numpy().reshape(-1)
    del plain, full
    z, y, x = np.meshgrid(*(np.arange(c0, c0 + size),) * 3, indexing="ij")
    pts = np.stack([x, y, z], -1).reshape(-1, 3)
    gt, lo, hi, ne, _ = gauss.prepare(w.gauss, [w.volume])[0]
    sel = ne & np.all(lo <= c0 + size - 1, 1) & np.all(hi >= c0, 1)
    gs = {k: gt[k][sel] for k in ("c", "C", "amp")}
    ref_g = gauss.render_points(pts, gs, lo[sel], hi[sel], ne[sel])
    xw = onrf.world_coords(pts, onrf.index_to_world(w.volume.world_to_index))
    r_ref, *_ = onrf.forward(net.weights_host(), onrf.encode(xw, 16, net.in_pad), net.out_scale)
    e32 = normwise(g_plain, ref_g)
    e_r = normwise(g_full - g_plain, r_ref)
    e_all = normwise(g_full, ref_g + r_ref)
    report("c320 crop [128,192)^3", "volume I (Gaussians)", "FP32", g_plain, ref_g)
    report("c320 crop [128,192)^3", "residual field r", "BF16 MFMA, FP32 acc.", g_full - g_plain,
           r_ref)
    report("c320 crop [128,192)^3", "I + r", "FP32 + BF16", g_full, ref_g + r_ref)
    say(f"  c320 crop: {int(sel.sum())} Gaussians meet it")
    say(f"  FP32 Gaussians: normwise {e32:.2e}, per-element {elementwise(g_plain, ref_g):.2e}")
    say(f"  BF16 field r: normwise {e_r:.2e}, per-element {elementwise(g_full - g_plain, r_ref):.2e}")
    say(f"  sum: normwise {e_all:.2e}, per-element {elementwise(g_full, ref_g + r_ref):.2e}")
    assert e32 <= TOL
    assert e_r <= TOL_BF16
    assert e_all <= TOL_BF16


def test_c256_fused_render_field_loss_equals_its_parts(mods):
    """The field-on training step's first pass at full size (1M Gaussians, three 256x256x64
    stacks, 12288 tiles: the loss finish's multi-round loop and every block of the fused
    kernel's resident grid): renderings and dL/dI bit for bit against render, the field's
    forward and the smooth-L1 called one after the other, the loss to 1e-6."""
    _lib, api, nrf = mods
    w = inputs.workload("c256", with_data=True, device="cuda")
    p = api.GaussParams.from_host(w.gauss)
    b = api.Bins(p.n, w.stacks, capacity=int(12 * p.n * len(w.stacks)))
    b.bin(p)
    ids = list(range(len(w.stacks)))
    targ = [d.contiguous() for d in w.stack_data]
    net = nrf.NRF(n_freq=16, depth=3, seed=0, zero_last=False)
    say("c256 fused render + field + loss against its parts")
    outs = api.render(b, ids)
    for k in ids:
        net.forward_add(w.stacks[k], outs[k])
    ref_loss, ref_dl = api.smooth_l1(outs, targ)
    stored = [torch.full(s.shape, float("nan"), device="cuda") for s in w.stacks]
    loss, dl = api.render_loss(b, ids, targ, outs=stored, nrf=net)
    torch.cuda.synchronize()
    for k in ids:
        assert torch.equal(stored[k], outs[k]), f"stack {k}: rendering + field differs"
        assert torch.equal(dl[k], ref_dl[k]), f"stack {k}: dL/dI differs"
    say(f"  loss {float(loss):.9g} against {float(ref_loss):.9g}")
    assert float(loss) == pytest.approx(float(ref_loss), rel=1e-6)


def test_c256_training_step_every_voxel_and_gaussian(mods):
    """The benchmark's training iteration on the 256^3 workload (1M Gaussians, three
    256x256x64 stacks: gm_bin, the render with the smooth-L1 epilogue over 12k tiles, the grid
    partials, the chain rule with Adam fused) against the oracle's FP64 iteration: every stack
    voxel, the loss, every dL/dI, and every Gaussian's new parameters and moments (Adam range
    of the gradient bar, as in test_gpu_train_step)."""
    from oracle import train
    _lib, api, _ = mods
    w = inputs.workload("c256", with_data=True)
    stacks = w.stacks
    targets = [np.asarray(d, np.float32) for d in w.stack_data]
    p = api.GaussParams.from_host(w.gauss)
    m = api.GaussParams.zeros_like(p)
    v = api.GaussParams.zeros_like(p)
    ids = list(range(len(stacks)))
    b = api.Bins(p.n, stacks, capacity=int(12 * p.n * len(stacks)))
    b.bin(p)
    tg = [torch.from_numpy(t).cuda() for t in targets]
    outs = [torch.empty(s.shape, device="cuda") for s in stacks]
    dls = [torch.empty(s.shape, device="cuda") for s in stacks]
    loss, _ = api.render_loss(b, ids, tg, dls, outs=outs)
    api.grid_partials(p, b, ids, dls)
    lrs = (1e-3, 1e-3, 5e-3, 5e-2)
    api.chain_adam(p, b, ids, m, v, lrs, 1, 0.1, 1.5)
    torch.cuda.synchronize()
    say(f"  c256 step: {b.n_pairs} (tile, Gaussian) pairs, {sum(b.box_pairs_host)} voxel pairs, "
        f"{b.total_tiles} tiles")
    params0 = [np.asarray(getattr(w.gauss, k), np.float32) for k in ("mean", "quat", "log_scale",
                                                                     "logit")]
    z = [np.zeros(a.shape, np.float32) for a in params0]
    ref = train.step(params0, z, z, 1, stacks, targets, lrs, 0.1, 1.5)
    for k, (o, r) in enumerate(zip(outs, ref["renders"])):
        o = o.cpu().numpy()
        e = normwise(o, r)
        report("c256 step", f"stack {k} I, every voxel", "FP32", o, r)
        say(f"  stack {k}: every voxel normwise {e:.2e}, per-element {elementwise(o, r):.2e}")
        assert e <= TOL
    report("c256 step", "smooth-L1 loss", "FP32 (FP64 sums)", [float(loss)], [ref["loss"]])
    say(f"  loss gpu {float(loss):.9g} oracle {ref['loss']:.9g}")
    assert abs(float(loss) - ref["loss"]) <= TOL * ref["loss"]
    for k, (d, r) in enumerate(zip(dls, ref["dl"])):
        e = normwise(d.cpu().numpy(), r)
        report("c256 step", f"dL/dI stack {k}", "FP32", d.cpu().numpy(), r)
        say(f"  dL/dI stack {k}: normwise {e:.2e}")
        assert e <= TOL
    gmax_s = np.max(np.abs(ref["grads"][2]))
    for k, (name, got_p, got_m, got_v) in enumerate(zip(("mean", "quat", "log_scale", "logit"),
                                                        p.tensors(), m.tensors(), v.tensors())):
        gref = ref["grads"][k]
        gmax = max(np.max(np.abs(gref)), gmax_s if name == "quat" else 0.0)
        delta = np.full(gref.shape, TOL * gmax)
        p_in = params0[k].astype(np.float64)
        rp, rm, rv = adam_range(p_in, gref, delta, z[k], z[k], 1, lrs[k])
        e_p = check_range(f"{name} p", got_p.cpu().numpy(), rp, ref["p"][k], p_in)
        e_m = check_range(f"{name} m", got_m.cpu().numpy(), rm, ref["m"][k], None)
        e_v = check_range(f"{name} v", got_v.cpu().numpy(), rv, ref["v"][k], None)
        # after Adam's first step m = (1 - beta1) g: the raw gradient of every Gaussian
        report("c256 step", f"dL/d{name} (Adam m / 0.1), every Gaussian", "FP32 (FP64 chain)",
               got_m.cpu().numpy() / 0.1, np.asarray(ref["grads"][k]))
        report("c256 step", f"{name} after Adam", "FP32", got_p.cpu().numpy(), ref["p"][k])
        say(f"  {name}: p {e_p:.2e} m {e_m:.2e} v {e_v:.2e} (normwise to the oracle)")

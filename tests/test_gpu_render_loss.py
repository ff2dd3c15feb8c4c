"""Fused render + smooth-L1 (gm_render_loss_smooth_l1) against the two-call path and the oracle.

Bars: dL/dI and the stored renderings bit-identical to gm_render_stacks followed by
gm_loss_smooth_l1 (same FP32 operations per voxel); the loss within 1e-6 relative of the
two-call path and of the oracle's FP64 smooth-L1 of the same renderings (only the order of
the FP64 sum differs); renderings within 1e-5 normwise of the oracle's.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import gauss
from paper_2603_00145_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    from paper_2603_00145_amd import api as _api
    _api.load()
    return _api


def problem(seed, n_g=600, n=37):
    rng = np.random.default_rng(seed)
    g = inputs.init_anisotropic(n, n_g, rng)
    grids = [inputs.stack_grid("axial", n, 11, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("coronal", n, 9, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("sagittal", n, 10, 1.0),
             inputs.volume_grid(n)]
    # targets around the renderings' range, so that |I - y| falls on both sides of beta = 1
    targ = [rng.normal(0.3, 1.0, size=gr.shape).astype(np.float32) for gr in grids]
    return g, grids, targ


@pytest.mark.parametrize("seed,ids", [(0, [0, 1, 2, 3]), (1, [3, 1]), (2, [2])])
def test_fused_equals_two_calls(api, seed, ids):
    g, grids, targ = problem(seed)
    say("render+loss seed", seed, "ids", ids)
    b = api.Bins(g.n, grids)
    b.bin(api.GaussParams.from_host(g))
    t = [torch.from_numpy(targ[i]).cuda() for i in ids]
    outs = api.render(b, ids)
    ref_loss, ref_dl = api.smooth_l1(outs, t)
    stored = [torch.full_like(o, float("nan")) for o in outs]
    loss, dl = api.render_loss(b, ids, t, outs=stored)
    loss2, dl2 = api.render_loss(b, ids, t)
    torch.cuda.synchronize()
    for k in range(len(ids)):
        assert torch.equal(stored[k], outs[k]), f"grid {ids[k]}: stored rendering differs"
        assert torch.equal(dl[k], ref_dl[k]), f"grid {ids[k]}: dL/dI differs"
        assert torch.equal(dl2[k], dl[k])
    assert float(loss2) == float(loss)          # bit-reproducible, with or without outs
    assert float(loss) == pytest.approx(float(ref_loss), rel=1e-6)
    # the oracle's FP64 smooth-L1 of the same renderings, and the oracle's renderings
    rv, rg = gauss.smooth_l1([o.cpu().numpy() for o in outs], [targ[i] for i in ids])
    say(f"  loss {float(loss):.9g} two-call {float(ref_loss):.9g} oracle {rv:.9g}")
    assert float(loss) == pytest.approx(rv, rel=1e-6)
    refs = gauss.render_all(g, [grids[i] for i in ids])
    for o, r in zip(outs, refs):
        d = np.max(np.abs(o.cpu().numpy().astype(np.float64) - r))
        assert d <= 1e-5 * np.max(np.abs(r))


def test_fused_c64_workload(api):
    """The 64^3 workload's three stacks against their simulated data."""
    w = inputs.workload("c64", with_data=True)
    ids = [0, 1, 2]
    say("render+loss c64")
    b = api.Bins(w.gauss.n, w.stacks)
    b.bin(api.GaussParams.from_host(w.gauss))
    t = [torch.from_numpy(np.ascontiguousarray(d, np.float32)).cuda() for d in w.stack_data]
    outs = api.render(b, ids)
    ref_loss, ref_dl = api.smooth_l1(outs, t)
    loss, dl = api.render_loss(b, ids, t)
    torch.cuda.synchronize()
    for k in ids:
        assert torch.equal(dl[k], ref_dl[k])
    assert float(loss) == pytest.approx(float(ref_loss), rel=1e-6)


def test_fused_no_gaussians_and_errors(api):
    grids = [inputs.volume_grid(20), inputs.stack_grid("axial", 20, 5, 1.0)]
    g = inputs.init_anisotropic(20, 1, np.random.default_rng(1)).subset(slice(0, 0))
    b = api.Bins(0, grids)
    b.bin(api.GaussParams.from_host(g))
    rng = np.random.default_rng(2)
    targ = [rng.normal(size=gr.shape).astype(np.float32) for gr in grids]
    t = [torch.from_numpy(x).cuda() for x in targ]
    loss, dl = api.render_loss(b, [0, 1], t)
    torch.cuda.synchronize()
    rv, rg = gauss.smooth_l1([np.zeros_like(x) for x in targ], targ)
    assert float(loss) == pytest.approx(rv, rel=1e-6)
    for a, r in zip(dl, rg):
        assert np.max(np.abs(a.cpu().numpy() - r)) <= 1e-6 * np.max(np.abs(r))
    from paper_2603_00145_amd import _lib
    with pytest.raises(_lib.GmError):
        api.render_loss(b, [], [])                           # no grid listed
    small = api.Bins(0, grids)
    small.loss_part = small.loss_part[:1]                    # workspace below 8 x tiles
    small.bin(api.GaussParams.from_host(g))
    with pytest.raises(_lib.GmError, match="workspace"):
        api.render_loss(small, [0, 1], t)

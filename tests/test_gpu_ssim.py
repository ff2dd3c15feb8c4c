"""SSIM term of the reconstruction loss (Eq. 10) on the GPU against the FP64 oracle: loss value
and gradient within 1e-5 normwise on ragged stacks (slices smaller than the window, exact tile
multiples, one-row slices) and on the 256^3 workload's stacks (value over every slice, gradient
on sampled slices); accumulation into dl_di; bit-reproducibility."""
import sys

import numpy as np
import pytest
import torch

from oracle import ssim as osim
from paper_2603_00145_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(gpu, ref):
    ref = np.asarray(ref, np.float64)
    s = np.max(np.abs(ref))
    d = np.max(np.abs(np.asarray(gpu, np.float64) - ref))
    return d / s if s > 0 else d


@pytest.fixture(scope="module")
def api():
    from paper_2603_00145_amd import api as a
    a.load()
    return a


def test_ssim_ragged_parity_and_accumulation(api):
    rng = np.random.default_rng(21)
    shapes = [(3, 37, 45), (2, 16, 32), (1, 7, 5), (2, 1, 70), (1, 48, 33)]
    pairs = [inputs.slice_pair(s, rng) for s in shapes]
    say(f"  ssim ragged: shapes {shapes}")
    dev = torch.device("cuda", 0)
    preds = [torch.from_numpy(p).to(dev) for p, _ in pairs]
    targs = [torch.from_numpy(t).to(dev) for _, t in pairs]
    dl = [torch.zeros_like(p) for p in preds]
    lam = 0.5
    loss = float(api.ssim_loss(preds, targs, dl, lam))
    ref_val, ref_g = osim.ssim_loss([p for p, _ in pairs], [t for _, t in pairs])
    say(f"  loss gpu {loss:.8f} oracle {ref_val:.8f}")
    assert abs(loss - ref_val) <= TOL * abs(ref_val)
    first = [d.clone() for d in dl]
    for k, (d, g) in enumerate(zip(dl, ref_g)):
        err = normwise(d.cpu().numpy(), lam * g)
        say(f"  stack {k} {shapes[k]}: gradient normwise {err:.2e}")
        assert err <= TOL
    # accumulation: a second call adds the same (deterministic) gradient again
    loss2 = float(api.ssim_loss(preds, targs, dl, lam))
    assert loss2 == loss
    for d, f in zip(dl, first):
        assert torch.equal(d, 2.0 * f)


def test_ssim_identical_and_empty(api):
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(22)
    p, _ = inputs.slice_pair((2, 20, 40), rng)
    x = torch.from_numpy(p).to(dev)
    dl = [torch.zeros_like(x)]
    loss = float(api.ssim_loss([x], [x.clone()], dl, 1.0))
    assert abs(loss) < 1e-6
    assert float(dl[0].abs().max()) < 1e-9
    # a stack with no voxels next to a regular one: the empty one is ignored
    e = torch.zeros((0, 8, 8), device=dev)
    dl2 = [torch.zeros_like(e), torch.zeros_like(x)]
    loss2 = float(api.ssim_loss([e, x], [e.clone(), x.clone()], dl2, 1.0))
    assert abs(loss2) < 1e-6


def test_ssim_c256_stacks(api):
    """The 256^3 workload's three 256x256x64 stacks in one call.  Sampled outputs the oracle
    computes one by one: the gradient on three slices per stack, and the SSIM sum of those
    slices (each also run alone, whose loss is 1 - its sum / its pixel count).  The full
    call's loss is the voxel-weighted mean of the single-slice losses of every slice."""
    w = inputs.workload("c256", with_data=True)
    rng = np.random.default_rng(23)
    targs = [np.asarray(d, np.float32) for d in w.stack_data]
    preds = [np.clip(0.9 * t + 0.05 + rng.normal(0, 0.01, t.shape), 0, 1).astype(np.float32)
             for t in targs]
    dev = torch.device("cuda", 0)
    tp = [torch.from_numpy(p).to(dev) for p in preds]
    tt = [torch.from_numpy(t).to(dev) for t in targs]
    dl = [torch.zeros_like(p) for p in tp]
    loss = float(api.ssim_loss(tp, tt, dl, 0.5))
    n = sum(p.size for p in preds)
    scratch = torch.zeros_like(tp[0][0:1])
    acc = 0.0
    for k, (p, t) in enumerate(zip(preds, targs)):
        npix = p.shape[1] * p.shape[2]
        for z in range(p.shape[0]):
            lz = float(api.ssim_loss([tp[k][z:z + 1]], [tt[k][z:z + 1]], [scratch], 0.0))
            acc += (1.0 - lz) * npix
            if z in (0, p.shape[0] // 2, p.shape[0] - 1):
                ssum, grad = osim.ssim_slice(p[z], t[z])
                err = normwise(dl[k][z].cpu().numpy(), -0.5 * grad / n)
                say(f"  c256 stack {k} slice {z}: gradient normwise {err:.2e}, "
                    f"slice loss gpu {lz:.8f} oracle {1 - ssum / npix:.8f}")
                assert err <= TOL
                assert abs(lz - (1 - ssum / npix)) <= TOL * abs(1 - ssum / npix)
    ref = 1.0 - acc / n
    say(f"  c256 loss {loss:.8f}, from the single-slice losses {ref:.8f}")
    assert abs(loss - ref) <= 2e-6 * abs(ref)


def test_reconstruction_with_ssim_term(api):
    """The paper's full reconstruction loss (smooth-L1 + 0.5 SSIM) drives the 64^3 workload: the
    SSIM of the rendered stacks improves and the volume PSNR rises."""
    from paper_2603_00145_amd import recon
    w = inputs.workload("c64", device="cuda")
    g = inputs.init_anisotropic(64, 20000, np.random.default_rng(0))
    cfg = recon.TrainConfig(n_iter=60, lambda_ssim=0.5)
    r = recon.Reconstruction(w.stacks, w.stack_data, api.GaussParams.from_host(g), cfg, w.volume,
                             w.phantom)

    def ssim_now():
        r.bins.bin(r.p)
        outs = api.render(r.bins, r.ids)
        scratch = [torch.zeros_like(o) for o in outs]
        return float(api.ssim_loss(outs, r.targets, scratch, 0.0))

    before = ssim_now()
    hist = r.run()
    after = ssim_now()
    say(f"  L_SSIM {before:.4f} -> {after:.4f}; psnr {hist[0]['psnr']:.2f} -> {hist[-1]['psnr']:.2f}")
    assert after < before
    assert hist[-1]["psnr"] > hist[0]["psnr"]

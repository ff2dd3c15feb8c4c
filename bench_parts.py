"""Throughput of the parts of the path outside the benchmark's iteration (neural residual field
and warm-start network against the dense BF16 MFMA peak; the SSIM loss term against the FP64
vector peak), each on its own, timed with HIP events on the launch stream.

    python bench_parts.py [--reps 10]

Prints one JSON line per measurement.  The algorithmic FLOP counts are the multiply-adds of
the layers as the kernels run them (inputs zero-padded to a multiple of 16 features):
    NRF forward, per point:   2 (in_pad*64 + (D-1)*64*64 + 64)
    NRF backward, per point:  forward recompute + dA (2 per weight of the hidden and input
                              layers but the first) + dW (2 per weight)
    SSIM value + gradient, per pixel: SSIM_FLOP_PER_PIXEL (FP64, against the FP64 peak)
    warm-start forward, per Gaussian: 2 * sum_l (c_out * K_pad,l * positions_out,l) + head
    warm-start training step: forward + backward-data (all but the first layer) + backward-
                              weights, i.e. about 3x forward.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from paper_2603_00145_amd import api, inputs, nrf, warmstart  # noqa: E402

BF16_PEAK = 2.5e15          # dense MFMA FLOP/s of MI355X in BF16
FP64_PEAK = 78.6e12         # FP64 vector FLOP/s of MI355X (an FMA counts 2)
HBM_PEAK = 8.0e12           # bytes/s
# SSIM value + gradient per pixel, separable 11-tap window: five window sums (2 x 11 FMA each)
# and three products, ~35 FLOP for the statistics and partials (plus two divisions), three
# adjoint window sums (2 x 11 FMA each) and 5 FLOP to assemble the gradient
SSIM_FLOP_PER_PIXEL = 2 * 5 * 22 + 3 + 35 + 2 * 3 * 22 + 5


def _time(fn, reps):
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def nrf_flops(net, backward=False):
    w = net.in_pad * 64 + (net.depth - 1) * 64 * 64 + 64
    fwd = 2 * w
    if not backward:
        return fwd
    da = 2 * ((net.depth - 1) * 64 * 64 + 64)    # dA through the hidden layers and head
    dw = 2 * w
    return fwd + da + dw


def warm_flops_forward():
    layers = [(32, 96, 512), (32, 864, 64), (32, 864, 8), (32, 256, 1)]   # c_out, K_pad, P_out
    return 2 * sum(c * k * p for c, k, p in layers) + 2 * 8 * 32


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--only", choices=["nrf", "ssim", "warm", "pose", "lattice"], default=None,
                    help="run one group of measurements")
    args = ap.parse_args()
    run = (lambda grp: args.only is None or args.only == grp)
    api.load()
    dev = torch.device("cuda", 0)
    out = []

    g = torch.Generator(device=dev)
    g.manual_seed(0)
    if run("nrf"):
        # NRF forward on the 256^3 volume and backward on 2^18 samples of each of three stacks
        w = inputs.workload("c256", with_data=False)
        net = nrf.NRF(n_freq=16, depth=3, seed=1, zero_last=False)
        vol = torch.zeros(w.volume.shape, dtype=torch.float32, device=dev)
        t = _time(lambda: net.forward_add(w.volume, vol), args.reps)
        pts = w.volume.n_voxels
        f = nrf_flops(net) * pts
        out.append({"what": "nrf_forward", "points": pts, "seconds": t, "points_per_s": pts / t,
                    "tflops": f / t / 1e12, "mfma_frac": f / t / BF16_PEAK,
                    "config": "L=16, in_pad 128, 3 x 64 SiLU, 256^3 voxel centres"})
        dl = torch.randn(w.stacks[0].shape, device=dev, generator=g)
        idx = torch.randint(0, w.stacks[0].n_voxels, (1 << 18,), device=dev, dtype=torch.int32,
                            generator=g)

        def nrf_bwd():
            net.zero_grad()
            net.backward_grids(w.stacks, [dl] * len(w.stacks), idxs=[idx] * len(w.stacks))
        t = _time(nrf_bwd, args.reps)
        pts = 3 * (1 << 18)
        f = nrf_flops(net, backward=True) * pts
        out.append({"what": "nrf_backward", "points": pts, "seconds": t, "points_per_s": pts / t,
                    "tflops": f / t / 1e12, "mfma_frac": f / t / BF16_PEAK,
                    "config": "2^18 sampled voxels on each of three 256x256x64 stacks"})

    if run("ssim"):
        # SSIM term (value + gradient) on three 256x256x64 stacks
        rng = np.random.default_rng(0)
        pairs = [inputs.slice_pair((64, 256, 256), rng) for _ in range(3)]
        sp = [torch.from_numpy(p).to(dev) for p, _ in pairs]
        st = [torch.from_numpy(q).to(dev) for _, q in pairs]
        sd = [torch.zeros_like(p) for p in sp]
        t = _time(lambda: api.ssim_loss(sp, st, sd, 0.5), args.reps)
        pix = sum(p.numel() for p in sp)
        f = SSIM_FLOP_PER_PIXEL * pix
        out.append({"what": "ssim_loss", "pixels": pix, "seconds": t, "pixels_per_s": pix / t,
                    "tflops_fp64": f / t / 1e12, "fp64_frac": f / t / FP64_PEAK,
                    "config": "three 256x256x64 stacks, 11x11 window, value + gradient, FP64"})

    if run("warm"):
        # warm-start network: inference on 256k Gaussians, one training step of batch 1024
        ws = warmstart.WarmStartNet(seed=0, zero_head=False)
        n = 1 << 18
        patches = torch.rand((n, 3, 512), device=dev, generator=g)
        patches = patches.to(torch.bfloat16).view(torch.int16).contiguous()
        s0 = torch.full((n, 3), -4.0, device=dev)
        l0 = torch.zeros(n, device=dev)
        t = _time(lambda: ws.forward(patches, s0, l0), args.reps)
        f = warm_flops_forward() * n
        out.append({"what": "warmstart_forward", "gaussians": n, "seconds": t, "gaussians_per_s": n / t,
                    "tflops": f / t / 1e12, "mfma_frac": f / t / BF16_PEAK,
                    "config": "3 x 8^3 BF16 patches, four 3D convs of width 32 + head"})
        b = 1024
        sig = warmstart.sym6(s0[:b] + 0.1, torch.tensor([[1.0, 0.1, 0.0, 0.0]], device=dev).repeat(b, 1))
        lt = torch.zeros(b, device=dev)
        t = _time(lambda: ws.backward(patches[:b].contiguous(), s0[:b].contiguous(), l0[:b].contiguous(),
                                      sig, lt), args.reps)
        f = 3 * warm_flops_forward() * b
        out.append({"what": "warmstart_train_step", "gaussians": b, "seconds": t,
                    "gaussians_per_s": b / t, "tflops": f / t / 1e12, "mfma_frac": f / t / BF16_PEAK,
                    "config": "batch 1024: forward, loss head, backward-data and backward-weights"})
    if run("pose"):
        # stack-pose gradient of the 256^3 workload (1M Gaussians, three stacks), after the
        # grid-frame partials of a random dL/dI
        w = inputs.workload("c256", with_data=False)
        p = api.GaussParams.from_host(w.gauss)
        ids = list(range(len(w.stacks)))
        b = api.Bins(p.n, w.stacks, capacity=int(12 * p.n * len(ids)))
        b.bin(p)
        dl = [torch.randn(s.shape, device=dev, generator=g) for s in w.stacks]
        api.grid_partials(p, b, ids, dl)
        t = _time(lambda: api.pose_grads(p, b, ids), args.reps)
        # per (Gaussian, grid): 44 B of parameters, 40 B of partials, 4 B tile count
        byt = p.n * len(ids) * (44 + 40 + 4)
        out.append({"what": "pose_grads", "gaussians": p.n, "grids": len(ids), "seconds": t,
                    "gb_per_s": byt / t / 1e9, "hbm_frac": byt / t / HBM_PEAK,
                    "config": "1M Gaussians x 3 stacks of 256x256x64, FP64 reduction"})

    if run("lattice"):
        # progressive-training transition 100^3 -> 126^3 lattices (1M -> 2M Gaussians)
        n0, n1 = 100, 126
        c = torch.linspace(-1 + 1 / n0, 1 - 1 / n0, n0, device=dev)
        Z, Y, X = torch.meshgrid(c, c, c, indexing="ij")
        m = torch.stack([X, Y, Z], -1).reshape(-1, 3).contiguous()
        p = api.GaussParams(m, torch.randn((n0 ** 3, 4), device=dev, generator=g),
                            torch.full((n0 ** 3, 3), -4.0, device=dev),
                            torch.randn(n0 ** 3, device=dev, generator=g))
        t = _time(lambda: api.upsample_lattice(p, n0, n1), args.reps)
        byt = n0 ** 3 * 32 + n1 ** 3 * 44      # old quat, scale, logit read; new lattice written
        out.append({"what": "upsample_lattice", "gaussians_out": n1 ** 3, "seconds": t,
                    "gb_per_s": byt / t / 1e9, "hbm_frac": byt / t / HBM_PEAK,
                    "config": "100^3 -> 126^3 lattice, binary64 interpolation"})

    for o in out:
        print(json.dumps(o))
        sys.stdout.flush()


if __name__ == "__main__":
    main()

"""Whole reconstructions of the synthetic workloads on one MI355X: wall time and ms per
iteration of a fit, PSNR of the rendered volume against the phantom before and after.

    python bench_fit.py --workload c128 --iters 200                       # 200 Adam iterations
    python bench_fit.py --workload c256 --iters 1000 --init devox --nrf   # 1000, field on half way
    python bench_fit.py --workload c320 --iters 1000 --init devox --nrf   # five stacks, 2M

Each fit runs the training loop of paper_2603_00145_amd.recon (bin, render + smooth-L1, backward
partials, chain rule + Adam; with --nrf the residual field is switched on at half the iterations
and fused into the render, its gradient taken on 2^18 sampled voxels per stack).  The timed
region is iterations 2..N (the first sizes the buffers and runs before the timer); the PSNR
evaluations (a volume render against the phantom) run before and after it.  --init devox starts from the paper's uniform lattice (126^3 for c320, 100^3 for
c256, 50^3 for c128), --init random from the workload's random anisotropic Gaussians.  Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from paper_2603_00145_amd import api, inputs, nrf, recon  # noqa: E402

DEVOX = {"c64": 32, "c128": 50, "c256": 100, "c320": 126}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c128")
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--init", choices=["random", "devox"], default="random")
    ap.add_argument("--nrf", action="store_true", help="field on from half the iterations")
    a = ap.parse_args()
    dev = torch.device("cuda", 0)
    t0 = time.time()
    w = inputs.workload(a.workload, with_data=True, device=dev)
    data = [d.contiguous() for d in w.stack_data]
    if a.init == "devox":
        p = api.devox_init(DEVOX[a.workload], w.stacks, data)
    else:
        p = api.GaussParams.from_host(w.gauss, dev)
    net = nrf.NRF(n_freq=16, depth=3, seed=0) if a.nrf else None
    cfg = recon.TrainConfig(n_iter=a.iters, nrf=net, nrf_start=0.5)
    r = recon.Reconstruction(w.stacks, data, p, cfg, w.volume, w.phantom)
    setup = time.time() - t0
    psnr0 = r.psnr()
    r.step()                  # the first iteration sizes the buffers; it is timed with the rest
    torch.cuda.synchronize()
    t = time.time()
    for _ in range(a.iters - 1):
        r.step()
    torch.cuda.synchronize()
    loop = time.time() - t
    psnr1 = r.psnr()
    torch.cuda.synchronize()
    out = {"workload": a.workload, "n_gauss": p.n,
           "stacks": [f"{g.nx}x{g.ny}x{g.nz}" for g in w.stacks], "init": a.init,
           "iterations": a.iters, "field": "on from iteration %d" % (a.iters // 2 + 1) if a.nrf
           else "off", "seconds_iterations_2_to_n": loop, "ms_per_iteration": 1e3 * loop / (a.iters - 1),
           "psnr_before": psnr0, "psnr_after": psnr1, "setup_seconds": setup}
    print(json.dumps(out))


if __name__ == "__main__":
    main()

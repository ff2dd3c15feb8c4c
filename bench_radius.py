"""The paper's block-radius trade-off (Sec. 4.4, Tab. 4) on a synthetic workload: reconstructions
with the cell-neighbourhood query (Eqs. 4-6) at block radii 3..7 (cells = the Gaussian lattice),
against the 3-sigma box, reporting final PSNR, milliseconds per iteration (HIP events) and the
contributing (Gaussian, voxel) pairs each query evaluates.

    python bench_radius.py [--iters 150] [--lattice 32] [--workload c64] [--radii 3,4,5,6,7]

One JSON line per configuration.  The 64^3 workload's stacks are axis-aligned (no rigid
offsets): the query's voxel sets are boxes.  The 128^3 workload's stacks are rigidly rotated,
where every voxel of a Gaussian's bounding box is tested against its cell block.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from paper_2603_00145_amd import api, inputs, recon  # noqa: E402


def run(rule, radius, lattice, iters, w, data):
    cfg = recon.TrainConfig(n_iter=iters, psnr_every=10 ** 9, block_radius=radius,
                            cell_resolution=lattice if radius > 0 else 0)
    p = api.devox_init(lattice, w.stacks, data)
    r = recon.Reconstruction(w.stacks, data, p, cfg, w.volume, w.phantom)
    start = r.psnr()
    for _ in range(5):
        r.step()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(iters - 5):
        r.step()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (iters - 5)
    return {"workload": w.name, "rule": rule, "block_radius": radius, "lattice": lattice,
            "iters": iters,
            "psnr_start": start, "psnr": r.psnr(), "ms_per_iter": ms,
            "pairs_per_iter": sum(r.bins.box_pairs_host)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=150)
    ap.add_argument("--lattice", type=int, default=32)
    ap.add_argument("--workload", default="c64")
    ap.add_argument("--radii", default="3,4,5,6,7")
    args = ap.parse_args()
    api.load()
    w = inputs.workload(args.workload, device="cuda")
    data = [torch.as_tensor(d) for d in w.stack_data]
    rows = [run("3-sigma box", 0, args.lattice, args.iters, w, data)]
    for radius in (int(x) for x in args.radii.split(",")):
        rows.append(run("block", radius, args.lattice, args.iters, w, data))
    for row in rows:
        print(json.dumps(row))
        sys.stdout.flush()


if __name__ == "__main__":
    main()

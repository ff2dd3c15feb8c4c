"""Benchmark: Magnetic-Gaussian reconstruction iterations on one MI355X.

One step = one training iteration of the plain method on the 256^3 workload: bin the 1M
Gaussians onto the three 256x256x64 thick-slice stacks, render the stacks, smooth-L1 loss and
its per-voxel gradient, backward to every Gaussian parameter (+ anisotropy regulariser), Adam
on the four parameter groups.  Inputs are resident in HBM before timing starts.

Prints one JSON line (see the keys below).  --gpus N with N > 1 is refused: this build runs
on a single GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gaussian·voxel evals/s fwd+bwd; ms/iter and iters-to-PSNR at 256^3 vs plain"
UNIT = "Gaussian·voxel evals/s"

# Algorithmic work per contributing (Gaussian, voxel) pair of the forward render: 3 SUB for
# delta, 3 MUL + 6 FMA for C delta, 1 MUL + 2 FMA for delta . C delta, 1 FMA to accumulate
# (FMA = 2 FLOP) = 25 FLOP, plus one exp2.  Backward recompute + 10 partial sums: 52 FLOP +
# one exp2.
FLOP_FWD = 25
FLOP_BWD = 52
# Published MI355X peaks: FP32 vector 157.3 TFLOP/s (an FMA counts 2; the figure assumes
# packed FP32, which this build never issues, so 78.6 TFLOP/s is the unpacked ceiling) and
# HBM3E 8 TB/s.
FP32_PEAK = 157.3e12
FP32_PEAK_UNPACKED = 78.6e12
# Transcendental rate (every pair takes one v_exp_f32): measured on this part with a scratch
# probe of independent v_exp_f32 chains at full occupancy.
EXP_RATE_MEASURED = 13.9e12
# VALU issue model (secondary): 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 39.3e12 lane-slots/s;
# the direct forward formula issues 16 non-transcendental instructions per pair, the backward
# 32, and one v_exp_f32 costs EXP_SLOTS issue slots: the lane-slot rate over the measured exp
# rate, 39.3e12 / 13.9e12 = 2.8.
LANE_OPS = 256 * 4 * 16 * 2.4e9
FWD_VALU_INSTR = 16
EXP_SLOTS = LANE_OPS / EXP_RATE_MEASURED


class TimingEvent:
    """A HIP event created with hipEventDisableSystemFence, on the HIP runtime torch loaded.
    Recording a default event ends with a system-scope cache writeback and invalidation (about
    5 us of idle GPU per record on this part); an event used only for timing does not need it,
    and its timestamps are the same."""
    FLAG = 0x20000000
    _hip = None

    @classmethod
    def runtime(cls):
        if cls._hip is None:
            import ctypes
            with open("/proc/self/maps") as f:
                path = next(ln.split()[-1] for ln in f if "libamdhip64" in ln)
            cls._hip = ctypes.CDLL(path)
        return cls._hip

    def __init__(self):
        import ctypes
        self._ct = ctypes
        self.ev = ctypes.c_void_p()
        rc = self.runtime().hipEventCreateWithFlags(ctypes.byref(self.ev), ctypes.c_uint(self.FLAG))
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")

    def record(self, stream):
        rc = self._hip.hipEventRecord(self.ev, self._ct.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def elapsed_time(self, end) -> float:
        ms = self._ct.c_float()
        rc = self._hip.hipEventElapsedTime(self._ct.byref(ms), self.ev, end.ev)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(ms.value)

    def __del__(self):
        if self._hip is not None and self.ev:
            self._hip.hipEventDestroy(self.ev)


def alu_peak_tflops(flop_per_pair, instr_per_pair):
    """Issue-model FLOP/s ceiling of a kernel whose every pair costs instr_per_pair VALU slots."""
    return LANE_OPS / instr_per_pair * flop_per_pair / 1e12


def pair_roof(flop_per_pair, exps_per_pair, p_f=FP32_PEAK, p_e=EXP_RATE_MEASURED):
    """Pairs/s ceiling when the FLOP run at p_f and the exps at p_e, one after the other on the
    same vector unit: R = 1 / (flop / p_f + exps / p_e)."""
    return 1.0 / (flop_per_pair / p_f + exps_per_pair / p_e)


def recorded_counters(kernel):
    """Per-launch VALU instruction counts of `kernel` from its committed counter summary
    (profiles/<kernel>_valu_c256.md), if taken on the kernel as built now, else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel.split('<')[0]}_valu_c256.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            key, _, val = line.partition(":")
            fields[key.strip()] = val.strip()
    if fields.get("kernel") != kernel:
        return None
    from bench_profile import kernel_digest
    now = kernel_digest(kernel)
    if now is None or now != fields.get("kernel_asm_sha256"):
        return None
    out = {}
    for k, v in fields.items():
        if k.startswith("SQ_"):
            out[k] = float(v)
    out["pairs_per_launch"] = float(fields.get("pairs_per_launch", "nan"))
    return out


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from its committed counter summary, if that summary
    was taken on the kernel as it is built now (the same gfx950 assembly digest), else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel.split('<')[0]}_traffic_c256.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            key, _, val = line.partition(":")
            if key in ("traffic_bytes", "kernel", "kernel_asm_sha256"):
                fields[key] = val.strip()
    if fields.get("kernel") != kernel:
        return None
    from bench_profile import kernel_digest
    now = kernel_digest(kernel)
    if now is None or now != fields.get("kernel_asm_sha256"):
        return None
    return float(fields["traffic_bytes"])


def recorded_iters_to_psnr():
    """The committed warm-start experiment's iterations-to-PSNR on the held-out 256^3
    phantoms (a separate, longer run; reported beside the throughput, not re-measured)."""
    import re
    path = os.path.join(ROOT, "profiles", "warmstart_iters_to_psnr_256.md")
    if not os.path.exists(path):
        return None
    txt = " ".join(open(path).read().split())
    m = re.search(r"reached the target on (\d+)/(\d+) phantoms; iterations to target: mean "
                  r"([0-9.]+), median ([0-9.]+) \(plain arm: (\d+)\)", txt)
    if not m:
        return None
    out = {"warm_mean": float(m.group(3)), "warm_median": float(m.group(4)),
           "plain": int(m.group(5)), "reached": f"{m.group(1)}/{m.group(2)}",
           "source": "profiles/warmstart_iters_to_psnr_256.md"}
    m = re.search(r"The offset arm reached it on (\d+)/(\d+)", txt)
    if m:
        out["offset_reached"] = f"{m.group(1)}/{m.group(2)}"
    return out


def live_iters_to_psnr():
    """The warm-start experiment at reduced size, measured in this run: the network trained on
    8 reconstructions of 128^3 phantoms (200 iterations each), then 2 held-out 256^3 phantoms
    (1M Gaussians) reconstructed for 500 iterations from the plain devoxelization, the
    constant-offset control and the network's initialisation; iterations to the plain arm's
    final PSNR (PSNR every 10 iterations)."""
    from paper_2603_00145_amd import warmstart
    t0 = time.time()
    r = warmstart.run_experiment(n_train=8, n_test=2, train_iters=200, test_iters=500,
                                 net_steps=400)
    cases = r["cases"]
    return {"what": "8 training phantoms at 128^3, 2 held-out at 256^3, 500 iterations per arm",
            "plain": 500,
            "warm": [c["warm_iters_to_target"] for c in cases],
            "offset": [c["offset_iters_to_target"] for c in cases],
            "plain_final_psnr": [round(c["plain_final_psnr"], 2) for c in cases],
            "warm_final_psnr": [round(c["warm_final_psnr"], 2) for c in cases],
            "seconds": time.time() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--unfused-loss", action="store_true",
                    help="render and smooth-L1 as two calls (the renderings go through HBM)")
    ap.add_argument("--unfused-adam", action="store_true",
                    help="chain rule into a gradient buffer, then Adam per group (four calls)")
    ap.add_argument("--cpu-sample-gauss", type=int, default=200000)
    ap.add_argument("--cpu-sample-gauss-1core", type=int, default=15000)
    ap.add_argument("--pairs-log", default="",
                    help="write the contributing pairs of every step (warm-up included) here")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the live (reduced) iterations-to-PSNR experiment")
    ap.add_argument("--nrf-steps", type=int, default=10,
                    help="also time this many iterations with the neural residual field on "
                         "(0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB before timing")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_00145_amd import api, inputs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.time()
    w = inputs.workload(args.workload, with_data=True, device=dev)
    stacks = w.stacks
    targets = [d.contiguous() for d in w.stack_data]
    p = api.GaussParams.from_host(w.gauss, dev)
    grads = api.GaussParams.zeros_like(p)
    m = api.GaussParams.zeros_like(p)
    v = api.GaussParams.zeros_like(p)
    bins = api.Bins(p.n, stacks, capacity=int(12 * p.n * len(stacks)))
    outs = [torch.empty(g.shape, dtype=torch.float32, device=dev) for g in stacks]
    dls = [torch.empty(g.shape, dtype=torch.float32, device=dev) for g in stacks]
    ids = list(range(len(stacks)))
    lrs = (1e-3, 1e-3, 5e-3, 5e-2)  # mean, quat (rotation), log_scale, logit (intensity)
    print(f"# setup {time.time() - t0:.1f}s: {p.n} Gaussians, stacks "
          f"{[g.shape for g in stacks]}", file=sys.stderr, flush=True)

    if args.calib_copy_mib > 0:
        # a plain streaming kernel of known traffic (reads N bytes, writes N bytes), for
        # scaling the HBM byte counters of a profile; torch's copy_ would go to a DMA engine
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # stage -> events; every stage is timed on the stream its kernels are launched on.  By
    # default "render" is the fused render + smooth-L1 call (the loss and dL/dI are formed in
    # the render's epilogue) and "chain" the fused chain rule + Adam call; with the unfused
    # options the separate calls get stages of their own ("loss": the smooth-L1 pass and/or the
    # gradient clear, "adam": the four Adam steps).
    fused_adam = not args.unfused_adam
    stages = ("bin", "render", "loss", "partials", "chain", "adam")
    if fused_adam and not args.unfused_loss:
        stages = ("bin", "render", "partials", "chain")
    elif fused_adam:
        stages = ("bin", "render", "loss", "partials", "chain")
    ev = {k: [] for k in stages}
    step_no = [0]
    pair_log = []
    all_pairs = []

    def step(e):
        # e: the step's events (created beforehand), or None for an untimed step
        s = torch.cuda.current_stream()
        record = e is not None
        k = [0]

        def mark(name):
            # closes the stage before `name` (or the step, for None) and opens `name`
            if record:
                e[k[0]].record(s)
                k[0] += 1

        mark("bin")
        bins.bin(p)
        all_pairs.append(sum(bins.box_pairs_host))
        if record:
            pair_log.append(sum(bins.box_pairs_host))   # reported by gm_bin, no extra sync
        mark("render")
        if args.unfused_loss:
            api.render(bins, ids, outs)                  # k_render
            mark("loss")
            loss, _ = api.smooth_l1(outs, targets, dls)
        else:
            loss, _ = api.render_loss(bins, ids, targets, dls)   # k_render, loss epilogue
            if not fused_adam:
                mark("loss")
        if not fused_adam:
            grads.zero_()
        mark("partials")
        api.grid_partials(p, bins, ids, dls)              # k_partials
        mark("chain")
        step_no[0] += 1
        if fused_adam:
            # k_chain (+ anisotropy) with Adam on the four groups in its epilogue
            api.chain_adam(p, bins, ids, m, v, lrs, step_no[0], 0.1, 1.5)
        else:
            api.chain(p, bins, ids, grads, 0.1, 1.5)      # k_chain (+ anisotropy)
            mark("adam")
            for prm, gr, mm, vv, lr in zip(p.tensors(), grads.tensors(), m.tensors(),
                                           v.tensors(), lrs):
                api.adam_step(prm, gr, mm, vv, lr, step_no[0])
        mark(None)
        return e, loss

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    recs = [[TimingEvent() for _ in range(len(stages) + 1)] for _ in range(args.steps)]
    start, stop = TimingEvent(), TimingEvent()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    start.record(stream)
    for e in recs:
        _, loss = step(e)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ms_step = total_ms / args.steps
    for e in recs:
        for k, (a, b) in zip(ev, zip(e[:-1], e[1:])):
            ev[k].append(a.elapsed_time(b))
    stage_ms = {k: float(np.mean(x)) for k, x in ev.items()}
    step_ms = np.array([e[0].elapsed_time(e[-1]) for e in recs])

    # contributing (Gaussian, voxel) pairs on the stacks, mean over the timed steps (the
    # Gaussians move, so the count changes from step to step)
    pairs = float(np.mean(pair_log))
    tile_pairs = bins.n_pairs
    value = sum(pair_log) / (total_ms / 1e3)
    bwd_ms = stage_ms["partials"] + stage_ms["chain"]
    fwd_rate = pairs / (stage_ms["render"] / 1e3)
    bwd_rate = pairs / (bwd_ms / 1e3)
    # The pair kernels' rooflines (one launch per step each; `roofline` is the dominant one):
    # algorithmic FLOP per launch (FLOP per contributing pair x the pairs gm_bin reported for
    # the step) over the stage's HIP-event time on the launch stream, against the published
    # FP32 peak.  The render stage also holds the 4-5 us one-block sum of the loss partials.
    def kernel_roofline(stage):
        if stage == "render":
            flop, instr, kname = FLOP_FWD, FWD_VALU_INSTR + EXP_SLOTS, "k_render"
        else:
            flop, instr, kname = FLOP_BWD, 2 * FWD_VALU_INSTR + EXP_SLOTS, "k_partials<false>"
        sec = stage_ms[stage] / 1e3
        achieved = flop * pairs / sec / 1e12
        peak = FP32_PEAK / 1e12
        r = {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": peak,
             "unit": "TFLOP/s", "frac": achieved / peak, "traffic": recorded_traffic(kname),
             "flop_per_pair": flop, "avg_kernel_ms": stage_ms[stage],
             "frac_of_unpacked_fp32": achieved * 1e12 / FP32_PEAK_UNPACKED,
             "issue_model": {"peak": alu_peak_tflops(flop, instr), "slots_per_pair": instr,
                             "frac": achieved / alu_peak_tflops(flop, instr)}}
        cnt = recorded_counters(kname)
        if cnt is not None:
            # every evaluated (Gaussian, voxel) lane takes one v_exp_f32; a wave instruction
            # covers 64 lanes, so contributing pairs / (64 x exp instructions) is the fraction of
            # evaluated lane-pairs that contribute (the per-piece log2 of the setup counts too,
            # so this slightly understates it)
            trans = cnt.get("SQ_INSTS_VALU_TRANS_F32")
            if trans:
                r["lane_efficiency"] = cnt["pairs_per_launch"] / (64.0 * trans)
                r["exp_lane_rate_per_s"] = 64.0 * trans / sec
                r["exp_lane_rate_frac_of_measured_peak"] = 64.0 * trans / sec / EXP_RATE_MEASURED
            fma = cnt.get("SQ_INSTS_VALU_FMA_F32")
            if fma is not None:
                r["fma_flop_rate_tflops"] = 2 * 64.0 * fma / sec / 1e12
            r["counters_per_launch"] = cnt
        return r

    dom = "render" if stage_ms["render"] >= stage_ms["partials"] else "partials"
    rooflines = {s: kernel_roofline(s) for s in ("render", "partials")}
    pair_ms = stage_ms["render"] + stage_ms["partials"]
    fb_rate = pairs / (pair_ms / 1e3)
    fwd_bwd_roof = {
        "what": "forward + backward pair rate (k_render + k_partials time) against "
                "R = 1/(77/P_F + 2/P_E): 77 FLOP and 2 exp per contributing pair",
        "achieved_pairs_per_s": fb_rate,
        "R_pairs_per_s": pair_roof(FLOP_FWD + FLOP_BWD, 2),
        "frac": fb_rate / pair_roof(FLOP_FWD + FLOP_BWD, 2),
        "R_unpacked_pairs_per_s": pair_roof(FLOP_FWD + FLOP_BWD, 2, FP32_PEAK_UNPACKED),
        "frac_unpacked": fb_rate / pair_roof(FLOP_FWD + FLOP_BWD, 2, FP32_PEAK_UNPACKED),
        "P_F": FP32_PEAK, "P_E": EXP_RATE_MEASURED,
        "achieved_tflops": (FLOP_FWD + FLOP_BWD) * fb_rate / 1e12,
        "frac_of_fp32_peak": (FLOP_FWD + FLOP_BWD) * fb_rate / FP32_PEAK,
        "whole_iteration_frac_of_fp32_peak":
            (FLOP_FWD + FLOP_BWD) * pairs / (ms_step / 1e3) / FP32_PEAK,
        "target": 0.5, "target_met": bool(fb_rate / pair_roof(FLOP_FWD + FLOP_BWD, 2) >= 0.5),
    }

    if args.pairs_log:
        with open(args.pairs_log, "w") as f:
            json.dump(all_pairs, f)

    nrf_on = None
    if args.nrf_steps > 0:
        nrf_on = time_nrf_on(args, bins, p, m, v, ids, stacks, targets, dls, lrs,
                             step_no[0])

    warm_live = None
    if not args.no_warm_start:
        warm_live = live_iters_to_psnr()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_sample_gauss, args.cpu_sample_gauss_1core)

    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w.n_vox}^3 phantom, {len(stacks)} stacks "
                   f"{'/'.join(f'{g.nx}x{g.ny}x{g.nz}' for g in stacks)} (thick slices, "
                   f"rigid offsets or oblique), {p.n} anisotropic Gaussians, plain method "
                   "(smooth-L1 + anisotropy, Adam)",
                   "n_gauss": p.n, "stacks": [list(g.shape) for g in stacks],
                   "tile": list(api._lib.tile_dims())},
        "ms_per_step_p10_p50_p90": [float(np.percentile(step_ms, q)) for q in (10, 50, 90)],
        "pairs_per_step": pairs, "tile_pairs": tile_pairs,
        "stage_ms": stage_ms, "fwd_evals_per_s": fwd_rate, "bwd_evals_per_s": bwd_rate,
        "fwd_bwd_evals_per_s": pairs / ((stage_ms["render"] + bwd_ms) / 1e3),
        "final_loss": float(loss),
        "loss_path": "two calls" if args.unfused_loss else "fused into the render",
        "adam_path": "four calls after the chain rule" if args.unfused_adam
                     else "fused into the chain rule (the chain stage includes Adam)",
        "roofline": rooflines[dom],
        "roofline_pair_kernels": {r["kernel"]: r for r in rooflines.values()},
        "roofline_fwd_bwd": fwd_bwd_roof,
        "cpu_baseline": cpu,
        "iters_to_psnr": {"measured_here": warm_live, "full_experiment": recorded_iters_to_psnr()},
        "nrf_on": nrf_on,
    }
    print(json.dumps(out))


def time_nrf_on(args, bins, p, m, v, ids, stacks, targets, dls, lrs, step0):
    """ms per iteration of the same workload with the neural residual field on (the second
    half of a reconstruction): bin, render + field + smooth-L1 in one pass, backward partials,
    the field's backward on 2^18 uniformly drawn voxels per stack (drawn beforehand: they are
    inputs), the field's Adam step, chain rule + Adam on the Gaussians."""
    import torch
    from paper_2603_00145_amd import api, nrf as nrfmod
    dev = p.mean.device
    net = nrfmod.NRF(n_freq=16, depth=3, seed=0, zero_last=False)
    n_sample = 1 << 18
    gen = torch.Generator(device=dev)
    gen.manual_seed(2603)
    total = args.nrf_steps + 2
    draws = [[torch.randint(0, g.n_voxels, (n_sample,), device=dev, dtype=torch.int32,
                            generator=gen) for g in stacks] for _ in range(total)]
    stages = ("bin", "render_field_loss", "partials", "field_backward", "chain")
    k_step = [step0]

    def step(i, e):
        s = torch.cuda.current_stream()
        k = [0]

        def mark():
            if e is not None:
                e[k[0]].record(s)
                k[0] += 1

        mark()
        bins.bin(p)
        mark()
        api.render_loss(bins, ids, targets, dls, nrf=net)
        mark()
        api.grid_partials(p, bins, ids, dls)
        mark()
        net.zero_grad()
        net.backward_grids(stacks, dls, idxs=draws[i])
        net.adam_step(1e-4)
        mark()
        k_step[0] += 1
        api.chain_adam(p, bins, ids, m, v, lrs, k_step[0], 0.1, 1.5)
        mark()

    for i in range(2):
        step(i, None)
    torch.cuda.synchronize()
    recs = [[TimingEvent() for _ in range(len(stages) + 1)] for _ in range(args.nrf_steps)]
    for i, e in enumerate(recs):
        step(i + 2, e)
    torch.cuda.synchronize()
    step_ms = np.array([e[0].elapsed_time(e[-1]) for e in recs])
    stage_ms = {st: float(np.mean([e[j].elapsed_time(e[j + 1]) for e in recs]))
                for j, st in enumerate(stages)}
    return {"what": "iteration with the residual field on (n_freq 16, 3 x 64, BF16 MFMA): "
                    "render + field + smooth-L1 fused, field backward on 2^18 sampled voxels "
                    "per stack, field and Gaussian Adam",
            "steps": args.nrf_steps, "ms_per_step": float(step_ms.mean()),
            "ms_per_step_p10_p50_p90": [float(np.percentile(step_ms, q)) for q in (10, 50, 90)],
            "stage_ms": stage_ms}


def cpu_baseline(w, n_gauss, n_gauss_1core):
    """The FP64 oracle, untuned, as a CPU reconstruction would run the same iteration: every
    Gaussian of a random sample scatters its values over its box on each stack (forward), then
    walks its box again for the ten partial sums and is pulled back through the chain rule
    (backward); contributing pairs per second, on every host core (OpenMP) and on one core (a
    smaller sample).  The FP64 per-Gaussian set-up (conic, amplitude, box) is excluded."""
    from oracle import gauss
    rng = np.random.default_rng(123)
    g = w.gauss
    dl = [np.asarray(d.cpu().numpy() if hasattr(d, "cpu") else d, np.float64) * 1e-6
          for d in w.stack_data]
    t_prep = time.time()
    prep = gauss.prepare(g, w.stacks)
    t_prep = time.time() - t_prep

    def run(n_sample):
        sub = np.sort(rng.choice(g.n, size=min(n_sample, g.n), replace=False))
        mean, quat, ls, logit = gauss.params64(g.subset(sub))
        pairs, t_f, t_b = 0, 0.0, 0.0
        parts = []
        for grid, (gt, lo, hi, ne, _), d in zip(w.stacks, prep, dl):
            gs = {k: (v[sub] if isinstance(v, np.ndarray) and v.shape[:1] == (g.n,) else v)
                  for k, v in gt.items() if k != "wt"}
            t = time.time()
            gauss.render_scatter(grid, gs, lo[sub], hi[sub], ne[sub])
            t_f += time.time() - t
            t = time.time()
            parts.append(gauss.grid_partials(grid, gs, lo[sub], hi[sub], ne[sub], d))
            t_b += time.time() - t
            pairs += int(np.where(ne[sub], np.prod(hi[sub] - lo[sub] + 1, axis=1), 0).sum())
        t = time.time()
        gauss.chain(mean, quat, ls, logit, w.stacks, parts)
        t_b += time.time() - t
        return pairs / (t_f + t_b), len(sub), pairs, t_f, t_b

    cores = gauss.threads()
    rate, n_all, p_all, tf_all, tb_all = run(n_gauss)
    gauss.set_threads(1)
    try:
        rate1, n_one, p_one, tf_one, tb_one = run(n_gauss_1core)
    finally:
        gauss.set_threads(cores)
    return {"value": rate, "unit": UNIT, "cores": cores, "kind": "oracle",
            "sample": f"FP64 box-scatter forward + box-walk backward + chain rule of {n_all} "
                      f"random Gaussians on the 3 stacks ({p_all} contributing pairs: forward "
                      f"{tf_all:.2f}s, backward {tb_all:.2f}s, {cores} threads); FP64 "
                      f"per-Gaussian set-up {t_prep:.1f}s excluded",
            "single_core": {"value": rate1, "cores": 1,
                            "sample": f"{n_one} random Gaussians ({p_one} pairs: forward "
                                      f"{tf_one:.2f}s, backward {tb_one:.2f}s)"}}


if __name__ == "__main__":
    main()

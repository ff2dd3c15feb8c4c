"""Training iterations exactly as Reconstruction.step() runs them (gm_bin -> fused render +
smooth-L1 -> grid partials -> fused chain rule + Adam; with the residual field on: render, the
field's forward added to the stacks, smooth-L1, its backward and Adam) against the FP64 oracle's
iteration (oracle/train.py), step by step, through the C ABI.

Before every step the GPU state (Gaussian parameters, Adam moments, the field's master weights
and moments) is set to the oracle's state after the previous step rounded to float32 (the seeded
initial state before the first), so both sides start each step from the same float32 values and
bin the same boxes; nothing the GPU computes flows into the oracle.

Bars.  The loss: 1e-5 relative.  Adam's update divides the first moment by the root of the
second, so near a zero gradient it turns rounding-level gradient differences into changes of
order the learning rate: a normwise 1e-5 bar on p, m, v cannot hold where the gradient is not
resolved.  Instead each output must lie in the image of the gradient bar under the oracle's
Adam step: the range of (p, m, v) over gradients g' in [g - d, g + d] elementwise (d the
gradient bar: 1e-5 of the tensor's largest gradient, the quaternion's taken against the
log-scale gradient for isotropic Gaussians), widened by 1e-5 of the update's (or moment's)
largest magnitude for FP32 arithmetic and by two float32 spacings of the stored value.  With
the residual field on, its BF16 outputs (2e-2 of max |r| per voxel) move dL/dI by at most
that / N per voxel, which moves each raw gradient by at most that times the sum over its boxes
of |d I / d theta| (oracle.gauss.abs_jacobian_sums): d is widened by it; the field's own
weights are held to the BF16 bar of its gradients (2e-2 normwise) through the same image.
"""
import sys

import numpy as np
import pytest
import torch

from adam_bounds import adam_range, check_range
from oracle import gauss, train
from paper_2603_00145_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-5
TOL_BF16 = 2e-2
LRS = (1e-3, 1e-3, 5e-3, 5e-2)
LAM_ANISO, LAM_R = 0.1, 1.5
GROUPS = ("mean", "quat", "log_scale", "logit")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    from paper_2603_00145_amd import api, nrf, recon
    api.load()
    return api, nrf, recon


def problem(case):
    if case == "ragged":
        rng = np.random.default_rng(21)
        n = 37
        g = inputs.init_anisotropic(n, 700, rng)
        stacks = [inputs.stack_grid("axial", n, 11, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
                  inputs.stack_grid("coronal", n, 9, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
                  inputs.stack_grid("sagittal", n, 10, 1.0)]
        targets = [rng.uniform(0, 1, size=s.shape).astype(np.float32) for s in stacks]
        return g, stacks, targets
    w = inputs.workload("c64")
    return w.gauss, w.stacks, [np.asarray(d, np.float32) for d in w.stack_data]


def field_init(depth, n_freq, in_pad, seed):
    """Seeded initial master weights in the kernels' layout; zero output layer (the field
    switches on continuously)."""
    rng = np.random.default_rng(seed)
    in_dim = 3 + 6 * n_freq
    w_in = np.zeros((64, in_pad), np.float32)
    w_in[:, :in_dim] = rng.uniform(-1, 1, (64, in_dim)) / np.sqrt(in_dim)
    return {"w_in": w_in, "b_in": (rng.uniform(-1, 1, 64) / np.sqrt(in_dim)).astype(np.float32),
            "w_hid": (rng.uniform(-1, 1, (max(depth - 1, 1), 64, 64)) / 8).astype(np.float32),
            "b_hid": (rng.uniform(-1, 1, (max(depth - 1, 1), 64)) / 8).astype(np.float32),
            "w_out": np.zeros(64, np.float32), "b_out": np.zeros(1, np.float32)}


@pytest.mark.parametrize("with_field", [False, True], ids=["plain", "field"])
@pytest.mark.parametrize("case", ["ragged", "c64"])
def test_training_steps_match_oracle(mods, case, with_field):
    api, nrf, recon = mods
    n_steps = 3
    g, stacks, targets = problem(case)
    say(f"case {case} field={with_field}: {g.n} Gaussians, stacks {[s.shape for s in stacks]}")
    net = None
    field = None
    if with_field:
        depth, n_freq = 3, 16
        net = nrf.NRF(n_freq=n_freq, depth=depth, seed=0)
        master = field_init(depth, n_freq, net.in_pad, seed=77)
        field = dict(master=master, m={k: np.zeros(v.shape, np.float32) for k, v in master.items()},
                     v={k: np.zeros(v.shape, np.float32) for k, v in master.items()}, t=1,
                     lr=1e-4, n_freq=n_freq, in_pad=net.in_pad, depth=depth,
                     out_scale=net.out_scale)
    cfg = recon.TrainConfig(n_iter=n_steps, lr_mean=LRS[0], lr_quat=LRS[1], lr_scale=LRS[2],
                            lr_logit=LRS[3], lambda_aniso=LAM_ANISO, lambda_r=LAM_R, nrf=net,
                            nrf_start=0.0, lr_nrf=1e-4)
    p = api.GaussParams.from_host(g)
    r = recon.Reconstruction(stacks, [torch.from_numpy(t).cuda() for t in targets], p, cfg)
    state_p = [np.asarray(getattr(g, k), np.float32) for k in GROUPS]
    state_m = [np.zeros(a.shape, np.float32) for a in state_p]
    state_v = [np.zeros(a.shape, np.float32) for a in state_p]
    ntot = sum(s.n_voxels for s in stacks)
    for t in range(1, n_steps + 1):
        # load the state into the GPU
        for dst, src in zip(r.p.tensors(), state_p):
            dst.copy_(torch.from_numpy(src))
        for dst, src in zip(r.m.tensors(), state_m):
            dst.copy_(torch.from_numpy(src))
        for dst, src in zip(r.v.tensors(), state_v):
            dst.copy_(torch.from_numpy(src))
        if with_field:
            for k in net.p:
                net.p[k].copy_(torch.from_numpy(field["master"][k]))
                net.m[k].copy_(torch.from_numpy(np.asarray(field["m"][k], np.float32)))
                net.v[k].copy_(torch.from_numpy(np.asarray(field["v"][k], np.float32)))
            net.step_no = t - 1
            net.sync_bf16()
            field["t"] = t
        assert r.it == t - 1
        say(f"  step {t}: GPU")
        loss_gpu = float(r.step())
        torch.cuda.synchronize()
        say(f"  step {t}: oracle")
        ref = train.step(state_p, state_m, state_v, t, stacks, targets, LRS, LAM_ANISO, LAM_R,
                         field)
        # loss
        extra = 0.0
        eps_r = 0.0
        if with_field:
            eps_r = TOL_BF16 * max(float(np.max(np.abs(x))) for x in ref["r"])
            extra = eps_r            # smooth-L1 is 1-Lipschitz per voxel; mean over voxels
        assert abs(loss_gpu - ref["loss"]) <= TOL * abs(ref["loss"]) + extra, \
            (loss_gpu, ref["loss"])
        # Gaussian groups
        A = gauss.abs_jacobian_sums(train._G(*state_p), stacks) if with_field else None
        got_p = [x.cpu().numpy() for x in r.p.tensors()]
        got_m = [x.cpu().numpy() for x in r.m.tensors()]
        got_v = [x.cpu().numpy() for x in r.v.tensors()]
        gmax_s = np.max(np.abs(ref["grads"][2]))
        for k, name in enumerate(GROUPS):
            gref = ref["grads"][k]
            gmax = np.max(np.abs(gref))
            if name == "quat":
                gmax = max(gmax, gmax_s)
            delta = np.full(gref.shape, TOL * gmax)
            if with_field:
                delta = delta + eps_r / ntot * A[k]
            p_in = state_p[k].astype(np.float64)
            rp, rm, rv = adam_range(p_in, gref, delta, state_m[k], state_v[k], t, LRS[k])
            e_p = check_range(f"step {t} {name} p", got_p[k], rp, ref["p"][k], p_in)
            e_m = check_range(f"step {t} {name} m", got_m[k], rm, ref["m"][k], None)
            e_v = check_range(f"step {t} {name} v", got_v[k], rv, ref["v"][k], None)
            say(f"    {name}: p {e_p:.2e} m {e_m:.2e} v {e_v:.2e} (normwise to the oracle)")
        if with_field:
            fp, fm, fv = ref["field"]
            for k in net.p:
                gk = np.asarray(ref["field_grads"][k], np.float64)
                delta = np.full(gk.shape, TOL_BF16 * max(np.max(np.abs(gk)), 1e-300))
                w0 = field["master"][k].astype(np.float64)
                rp, rm, rv = adam_range(w0, gk, delta, field["m"][k], field["v"][k], t, field["lr"])
                e_p = check_range(f"step {t} field {k} p", net.p[k].cpu().numpy(), rp, fp[k], w0)
                check_range(f"step {t} field {k} m", net.m[k].cpu().numpy(), rm, fm[k], None)
                check_range(f"step {t} field {k} v", net.v[k].cpu().numpy(), rv, fv[k], None)
                say(f"    field {k}: p {e_p:.2e}")
            field["master"] = {k: fp[k].astype(np.float32) for k in fp}
            field["m"] = {k: fm[k].astype(np.float32) for k in fm}
            field["v"] = {k: fv[k].astype(np.float32) for k in fv}
        say(f"    loss gpu {loss_gpu:.9g} oracle {ref['loss']:.9g}")
        state_p = [x.astype(np.float32) for x in ref["p"]]
        state_m = [x.astype(np.float32) for x in ref["m"]]
        state_v = [x.astype(np.float32) for x in ref["v"]]

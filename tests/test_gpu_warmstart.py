"""Warm-start network on MFMA against the FP64 oracle (same BF16-valued weights): patch
gather, forward outputs and every weight gradient, bar 2e-2 normwise; and a short training run
reduces its loss."""
import sys

import numpy as np
import pytest
import torch

from oracle import warm as owarm
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
    from paper_2603_00145_amd import api, warmstart
    api.load()
    return api, warmstart


def bf16_to_f64(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def test_gather_matches_oracle(mods):
    api, ws = mods
    w = inputs.workload("c64")
    rng = np.random.default_rng(0)
    means = rng.uniform(-0.9, 0.9, (32, 3)).astype(np.float32)
    got = ws.WarmStartNet.gather(w.stacks, [torch.from_numpy(d).cuda() for d in w.stack_data],
                                 torch.from_numpy(means).cuda(), 2.0 / 64)
    ref = owarm.gather(w.stacks, w.stack_data, means, 2.0 / 64).reshape(32, 3, 512)
    assert normwise(bf16_to_f64(got), ref) <= TOL_BF16


def test_targets_match_oracle(mods):
    """gm_ws_targets: training-target covariances against the oracle's FP64 covariance."""
    api, ws = mods
    rng = np.random.default_rng(4)
    n = 1000
    s = rng.normal(-3.5, 0.4, (n, 3)).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    got = ws.sym6(torch.from_numpy(s).cuda(), torch.from_numpy(q).cuda()).cpu().numpy()
    S = owarm.covariance(s.astype(np.float64), q.astype(np.float64))
    ref = np.stack([S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1], S[:, 0, 2], S[:, 1, 2]], 1)
    assert normwise(got, ref) <= 1e-6


@pytest.mark.parametrize("n", [48, 1024])
def test_forward_and_gradients_match_oracle(mods, n):
    """n = 1024 is the training batch: the head's weight gradient is then split over 64
    sample ranges and the convolution weight gradients over many sample partials."""
    api, ws = mods
    rng = np.random.default_rng(1)
    net = ws.WarmStartNet(seed=3, zero_head=False)
    X = rng.uniform(0, 1, (n, 3, 512)).astype(np.float32)
    Xb = torch.from_numpy(X).cuda().to(torch.bfloat16).view(torch.int16)
    s0 = rng.normal(-3.5, 0.1, (n, 3)).astype(np.float32)
    l0 = rng.normal(0, 0.5, n).astype(np.float32)
    s_t = rng.normal(-3.5, 0.3, (n, 3))
    q_t = rng.normal(size=(n, 4))
    sig = owarm.covariance(s_t, q_t)
    sig6 = np.stack([sig[:, 0, 0], sig[:, 1, 1], sig[:, 2, 2], sig[:, 0, 1], sig[:, 0, 2], sig[:, 1, 2]], 1)
    lt = rng.normal(size=n)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    s, q, lg = net.forward(Xb, T(s0), T(l0))
    loss = net.backward(Xb, T(s0), T(l0), T(sig6), T(lt))
    torch.cuda.synchronize()
    W = net.weights_host()
    X0 = bf16_to_f64(Xb).reshape(n, 3, 8, 8, 8)
    out, _, _ = owarm.forward(W, X0)
    rs, rq, rl = owarm.assemble(out, s0.astype(np.float64), l0.astype(np.float64))
    for name, a, r in (("log_scale", s, rs), ("quat", q, rq), ("logit", lg, rl)):
        err = normwise(a.cpu().numpy(), r)
        report(f"warm-start batch {n}", f"network output {name}", "BF16 MFMA, FP32 acc.",
               a.cpu().numpy(), r)
        say(f"  warm forward {name}: {err:.2e}")
        assert err <= TOL_BF16
    L, dout = owarm.loss_grad(out, s0.astype(np.float64), l0.astype(np.float64), sig, lt)
    assert float(loss) == pytest.approx(L, rel=TOL_BF16)
    g = owarm.backward(W, X0, dout)
    got = {f"W{l + 1}": net.g[f"w{l}"].cpu().numpy()[:, :ws.KREAL[l]] for l in range(4)}
    got.update({f"b{l + 1}": net.g[f"b{l}"].cpu().numpy() for l in range(4)})
    got["Wl"] = net.g["wl"].cpu().numpy()
    got["bl"] = net.g["bl"].cpu().numpy()
    for k in got:
        err = normwise(got[k], g[k].reshape(got[k].shape))
        report(f"warm-start batch {n}", f"weight gradient {k}", "BF16 MFMA, FP32 acc.", got[k],
               g[k].reshape(got[k].shape))
        say(f"  warm gradient {k}: {err:.2e}")
        assert err <= TOL_BF16, k


def test_chunked_inference_sampled(mods):
    """Inference as the warm start runs it, in chunks of 65536 Gaussians (two chunks, the second
    ragged): outputs at samples spread over both chunks and their edges against the oracle's
    forward of those samples (each sample's output depends on its own patch only)."""
    api, ws = mods
    rng = np.random.default_rng(6)
    n = (1 << 16) + 16 * 37
    net = ws.WarmStartNet(seed=5, zero_head=False)
    X = torch.rand((n, 3, 512), device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    Xb = X.to(torch.bfloat16).view(torch.int16)
    s0 = torch.from_numpy(rng.normal(-3.5, 0.1, (n, 3)).astype(np.float32)).cuda()
    l0 = torch.from_numpy(rng.normal(0, 0.5, n).astype(np.float32)).cuda()
    s, q, lg = net.forward(Xb, s0, l0)
    torch.cuda.synchronize()
    c = 1 << 16
    pick = np.unique(np.concatenate([np.arange(8), np.arange(c - 8, c + 8), np.arange(n - 8, n),
                                     rng.integers(0, n, 40)]))
    W = net.weights_host()
    X0 = bf16_to_f64(Xb[torch.from_numpy(pick).cuda()]).reshape(pick.size, 3, 8, 8, 8)
    out, _, _ = owarm.forward(W, X0)
    rs, rq, rl = owarm.assemble(out, s0.cpu().numpy()[pick].astype(np.float64),
                                l0.cpu().numpy()[pick].astype(np.float64))
    for name, a, r in (("log_scale", s, rs), ("quat", q, rq), ("logit", lg, rl)):
        err = normwise(a.cpu().numpy()[pick], r)
        say(f"  warm inference (chunked, {n}) {name}: {err:.2e} on {pick.size} samples")
        assert err <= TOL_BF16


def test_training_reduces_loss(mods):
    api, ws = mods
    rng = np.random.default_rng(2)
    n = 256
    net = ws.WarmStartNet(seed=0)
    X = torch.from_numpy(rng.uniform(0, 1, (n, 3, 512)).astype(np.float32)).cuda()
    Xb = X.to(torch.bfloat16).view(torch.int16)
    s0 = torch.full((n, 3), -3.5, device="cuda")
    l0 = torch.zeros(n, device="cuda")
    # targets that depend on the patch mean: learnable
    m = X.mean(dim=(1, 2))
    s_t = (-3.5 + 0.5 * (m - 0.5)).double()[:, None].repeat(1, 3)
    q_t = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    q_t[:, 0] = 1
    sig6 = ws.sym6(s_t, q_t).float().contiguous()
    lt = (2 * (m - 0.5)).contiguous()
    first = None
    for it in range(200):
        loss = float(net.train_step(Xb, s0, l0, sig6, lt, lr=3e-3))
        first = loss if first is None else first
    say(f"  warm training loss {first:.4f} -> {loss:.4f}")
    assert loss < 0.5 * first


def test_warm_start_gain_small(mods):
    """The iterations-to-PSNR experiment at small scale: a network trained on four 128^3
    reconstructions warm-starts a held-out 256^3 phantom, which then reaches the plain arm's
    200-iteration PSNR in at most half the iterations, and before the control arm (the best
    constant log-scale and logit offsets fitted on the same reconstructions) does."""
    from paper_2603_00145_amd import warmstart
    res = warmstart.run_experiment(n_train=4, n_test=1, train_iters=100, test_iters=200,
                                   net_steps=300)
    case = res["cases"][0]
    say(f"  plain {case['plain_init_psnr']:.2f} -> {case['plain_final_psnr']:.2f} dB; offset "
        f"{case['offset_init_psnr']:.2f} -> {case['offset_final_psnr']:.2f} dB (target at "
        f"{case['offset_iters_to_target']}); warm {case['warm_init_psnr']:.2f} -> "
        f"{case['warm_final_psnr']:.2f} dB (target at {case['warm_iters_to_target']}); offsets "
        f"{res['constant_offsets']}")
    assert res["net_loss"][-1][1] < res["net_loss"][0][1]
    assert case["warm_iters_to_target"] is not None
    assert case["warm_iters_to_target"] <= 100
    # the network does better than the best one-number fix learned from the same training set
    off = case["offset_iters_to_target"]
    assert off is None or case["warm_iters_to_target"] < off

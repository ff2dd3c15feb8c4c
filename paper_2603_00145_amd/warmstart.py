"""Learned warm start: a small 3D convolutional network that predicts, for each Gaussian of a
devoxelization initialisation, residuals of its log-scale, rotation and intensity from an 8^3
patch of the registered stacks (kernels in csrc/warm.hip), its training on reconstructions
produced by the plain method, and the iterations-to-PSNR comparison against the plain
devoxelization initialisation.
"""
from __future__ import annotations

import ctypes
import json
import math
import sys
import time
from typing import List, Optional

import numpy as np
import torch

from . import _lib, api, inputs, recon
from ._lib import check, load

KREAL = [81, 864, 864, 256]
KPAD = [96, 864, 864, 256]
SHAPES = [(32, 3, 3), (32, 32, 3), (32, 32, 3), (32, 32, 2)]  # (out, in, k)


class WarmStartNet:
    def __init__(self, seed: int = 0, zero_head: bool = True, device="cuda"):
        dev = torch.device(device)
        rng = np.random.default_rng(seed)
        p = {}
        for l in range(4):
            w = np.zeros((32, KPAD[l]), np.float32)
            b = 1.0 / math.sqrt(KREAL[l])
            w[:, :KREAL[l]] = rng.uniform(-b, b, (32, KREAL[l]))
            p[f"w{l}"] = w
            p[f"b{l}"] = rng.uniform(-b, b, 32).astype(np.float32)
        b = 1.0 / math.sqrt(32)
        p["wl"] = np.zeros((8, 32), np.float32) if zero_head else rng.uniform(-b, b, (8, 32)).astype(np.float32)
        p["bl"] = np.zeros(8, np.float32)
        self.p = {k: torch.from_numpy(v).to(dev).contiguous() for k, v in p.items()}
        self.g = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.bf = {f"w{l}": torch.empty((32, KPAD[l]), dtype=torch.int16, device=dev) for l in range(4)}
        self.step_no = 0
        self._ws = None
        self.sync_bf16()

    def sync_bf16(self):
        for k, t in self.bf.items():
            check(load().gm_f32_to_bf16(ctypes.c_void_p(self.p[k].data_ptr()),
                                        ctypes.c_void_p(t.data_ptr()), t.numel(), api._stream()))

    def struct(self):
        s = _lib.GmWsNet()
        for l in range(4):
            s.w[l] = self.bf[f"w{l}"].data_ptr()
            s.b[l] = self.p[f"b{l}"].data_ptr()
        s.wl, s.bl = self.p["wl"].data_ptr(), self.p["bl"].data_ptr()
        self._s = s
        return s

    def grads_struct(self):
        s = _lib.GmWsGrads()
        for l in range(4):
            s.w[l] = self.g[f"w{l}"].data_ptr()
            s.b[l] = self.g[f"b{l}"].data_ptr()
        s.wl, s.bl = self.g["wl"].data_ptr(), self.g["bl"].data_ptr()
        return s

    def _workspace(self, n, dev):
        nb = ctypes.c_size_t()
        check(load().gm_ws_workspace(n, ctypes.byref(nb)))
        if self._ws is None or self._ws.numel() * 4 < nb.value:
            self._ws = torch.empty((nb.value + 3) // 4, dtype=torch.float32, device=dev)
        return self._ws

    @staticmethod
    def gather(stacks, stack_data, means: torch.Tensor, spacing: float) -> torch.Tensor:
        n = means.shape[0]
        out = torch.empty((n, 3, 512), dtype=torch.int16, device=means.device)
        cg = (_lib.GmGrid * 3)(*[_lib.grid_struct(s) for s in stacks])
        check(load().gm_ws_gather(cg, 3, _lib.ptr_array([d.data_ptr() for d in stack_data]),
                                  ctypes.c_void_p(means.contiguous().data_ptr()), n, float(spacing),
                                  ctypes.c_void_p(out.data_ptr()), api._stream()))
        return out

    def forward(self, patches, s0, logit0, chunk: int = 1 << 16):
        """(log_scale, quat, logit) for a batch (n a multiple of 16), in chunks of `chunk`
        Gaussians so that the activation workspace stays bounded."""
        n = patches.shape[0]
        dev = patches.device
        s = torch.empty((n, 3), device=dev)
        q = torch.empty((n, 4), device=dev)
        lg = torch.empty((n,), device=dev)
        ws = self._workspace(min(n, chunk), dev)
        P = ctypes.c_void_p
        st = self.struct()
        for i0 in range(0, n, chunk):
            m = min(chunk, n - i0)
            check(load().gm_ws_forward(ctypes.byref(st), P(patches[i0].data_ptr()), m,
                                       P(s0[i0].data_ptr()), P(logit0[i0:].data_ptr()),
                                       P(s[i0].data_ptr()), P(q[i0].data_ptr()),
                                       P(lg[i0:].data_ptr()), P(ws.data_ptr()), ws.numel() * 4,
                                       api._stream()))
        return s, q, lg

    def backward(self, patches, s0, logit0, sig_t, logit_t):
        n = patches.shape[0]
        dev = patches.device
        loss = torch.empty(4, device=dev)
        ws = self._workspace(n, dev)
        P = ctypes.c_void_p
        gs = self.grads_struct()
        check(load().gm_ws_backward(ctypes.byref(self.struct()), P(patches.data_ptr()), n,
                                    P(s0.data_ptr()), P(logit0.data_ptr()), P(sig_t.data_ptr()),
                                    P(logit_t.data_ptr()), P(loss.data_ptr()), ctypes.byref(gs),
                                    P(ws.data_ptr()), ws.numel() * 4, api._stream()))
        return loss[0]

    def train_step(self, patches, s0, logit0, sig_t, logit_t, lr=1e-3):
        for t in self.g.values():
            t.zero_()
        loss = self.backward(patches, s0, logit0, sig_t, logit_t)
        self.step_no += 1
        for k in self.p:
            api.adam_step(self.p[k], self.g[k], self.m[k], self.v[k], lr, self.step_no)
        self.sync_bf16()
        return loss

    def weights_host(self):
        """BF16-valued conv weights [O, C, k, k, k] and FP32 head, float64 (for the oracle)."""
        net = {}
        for l, (o, c, k) in enumerate(SHAPES):
            u = self.bf[f"w{l}"].cpu().numpy().view(np.uint16).astype(np.uint32) << 16
            w = u.view(np.float32).astype(np.float64)[:, :KREAL[l]]
            net[f"W{l + 1}"] = w.reshape(o, c, k, k, k)
            net[f"b{l + 1}"] = self.p[f"b{l}"].cpu().numpy().astype(np.float64)
        net["Wl"] = self.p["wl"].cpu().numpy().astype(np.float64)
        net["bl"] = self.p["bl"].cpu().numpy().astype(np.float64)
        return net


def sym6(s: torch.Tensor, q: torch.Tensor) -> torch.Tensor:
    """Covariance (xx, yy, zz, xy, xz, yz) of log-scales s [n,3] and quaternions q [n,4]
    (gm_ws_targets): the warm-start training targets."""
    s = s.float().contiguous()
    q = q.float().contiguous()
    out = torch.empty((s.shape[0], 6), dtype=torch.float32, device=s.device)
    check(load().gm_ws_targets(ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                               s.shape[0], ctypes.c_void_p(out.data_ptr()), api._stream()))
    return out


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def make_case(n_vox, n_slices, seed, device, bias=True, n_ell=None):
    """Phantom, three rigidly offset orthogonal stacks (4x thicker slices) and their data."""
    ss = np.random.SeedSequence(seed)
    r_ph, r_st, r_noise = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
    stacks = inputs.orthogonal_stacks(n_vox, n_slices, 1.0, r_st, 2.0, 1.0)
    ph = inputs.make_phantom(n_vox, n_ell or max(12, n_vox // 3), r_ph, bias=bias, device=device)
    data = [inputs.simulate_stack(ph, s, r_noise, 0.01) for s in stacks]
    return stacks, data, ph, inputs.volume_grid(n_vox)


def constant_offsets(s0: torch.Tensor, l0: torch.Tensor, sig_t: torch.Tensor,
                     logit_t: torch.Tensor):
    """The control arm's fix: one log-scale offset d (added to all three log-scales) and one
    logit offset e, fitted on the training set in the network's own loss.  The devoxelization
    Gaussians are isotropic, Sigma0 = u0 I, so with u = u0 e^{2 d} the covariance term
    sum_i |u I - Sigma*_i|_F^2 / |Sigma*_i|_F^2 is a quadratic in u, least at
    u = sum_i tr(Sigma*_i) / |Sigma*_i|^2 / (3 sum_i 1 / |Sigma*_i|^2); the logit term is least at
    e = mean(logit* - logit0).  Returns (d, e) relative to each Gaussian's own initial values,
    so they transfer to a finer lattice as a ratio of scales."""
    S = sig_t.double().cpu().numpy()
    tr = S[:, 0] + S[:, 1] + S[:, 2]
    nrm = (S[:, :3] ** 2).sum(1) + 2.0 * (S[:, 3:] ** 2).sum(1)
    u = float(np.sum(tr / nrm) / (3.0 * np.sum(1.0 / nrm)))
    s0h = s0.double().cpu().numpy()
    u0 = np.exp(2.0 * s0h[:, 0])          # isotropic: the three log-scales are equal
    if not np.allclose(s0h, s0h[:, :1]) or not np.allclose(u0, u0[0]):
        raise ValueError("the constant-offset arm expects one isotropic initial scale")
    d = 0.5 * np.log(u / u0[0])
    e = float(np.mean(logit_t.double().cpu().numpy() - l0.double().cpu().numpy()))
    return float(d), e


def run_experiment(n_train=64, n_test=16, train_vox=128, test_vox=256, g_train=50, g_test=100,
                   train_iters=200, test_iters=1000, net_steps=1500, batch=1024, lr=1e-3,
                   psnr_every=10, device="cuda", out: Optional[str] = None):
    """Train the warm-start network on reconstructions of n_train phantoms (plain method from
    the devoxelization initialisation), then reconstruct n_test held-out phantoms from three
    initialisations - plain devoxelization, devoxelization with the best constant log-scale and
    logit offsets on the same training set (the control arm: what a one-number fix gains), and
    the network's - and compare iterations to the plain arm's final PSNR."""
    t0 = time.time()
    dev = torch.device(device)
    # 1. training reconstructions
    pats, s0s, l0s, sigs, lts = [], [], [], [], []
    h = 2.0 / g_train
    for i in range(n_train):
        stacks, data, ph, vol = make_case(train_vox, train_vox // 4, 4000 + i, dev)
        p0 = api.devox_init(g_train, stacks, data)
        init_s = p0.log_scale.clone()
        init_l = p0.logit.clone()
        r = recon.Reconstruction(stacks, data, p0, recon.TrainConfig(n_iter=train_iters), vol, None)
        for _ in range(train_iters):
            r.step()
        pats.append(WarmStartNet.gather(stacks, data, r.p.mean, h / 4))
        s0s.append(init_s)
        l0s.append(init_l)
        sigs.append(sym6(r.p.log_scale, r.p.quat))
        lts.append(r.p.logit.clone())
        _say(f"# train case {i + 1}/{n_train} done ({time.time() - t0:.0f}s)")
    P = torch.cat(pats)
    S0 = torch.cat(s0s)
    L0 = torch.cat(l0s)
    SIG = torch.cat(sigs)
    LT = torch.cat(lts)
    # 2. train the network
    net = WarmStartNet(seed=0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    losses = []
    for it in range(net_steps):
        idx = torch.randint(0, P.shape[0], (batch,), device=dev, generator=gen)
        loss = net.train_step(P[idx].contiguous(), S0[idx].contiguous(), L0[idx].contiguous(),
                              SIG[idx].contiguous(), LT[idx].contiguous(), lr)
        if it % 100 == 0 or it == net_steps - 1:
            losses.append((it, float(loss)))
            _say(f"# net step {it}: loss {float(loss):.4f} ({time.time() - t0:.0f}s)")
    del P
    d_off, e_off = constant_offsets(S0, L0, SIG, LT)
    _say(f"# constant offsets: log-scale {d_off:+.4f}, logit {e_off:+.4f}")
    # 3. held-out comparison
    h_t = 2.0 / g_test
    results = []
    for i in range(n_test):
        stacks, data, ph, vol = make_case(test_vox, test_vox // 4, 4100 + i, dev)
        arms = {}
        for arm in ("plain", "offset", "warm"):
            p0 = api.devox_init(g_test, stacks, data)
            if arm == "offset":
                p0 = api.GaussParams(p0.mean, p0.quat, (p0.log_scale + d_off).contiguous(),
                                     (p0.logit + e_off).contiguous())
            if arm == "warm":
                n = p0.n
                npad = (n + 15) // 16 * 16
                pad = lambda t: torch.cat([t, t[:npad - n]]) if npad > n else t
                pt = WarmStartNet.gather(stacks, data, pad(p0.mean).contiguous(), h_t / 4)
                s, q, lg = net.forward(pt, pad(p0.log_scale).contiguous(), pad(p0.logit).contiguous())
                p0 = api.GaussParams(p0.mean, q[:n].contiguous(), s[:n].contiguous(), lg[:n].contiguous())
            r = recon.Reconstruction(stacks, data, p0, recon.TrainConfig(n_iter=test_iters,
                                                                         psnr_every=psnr_every), vol, ph)
            hist = r.run()
            arms[arm] = hist
            _say(f"# test case {i + 1}/{n_test} {arm}: psnr {hist[0]['psnr']:.2f} -> "
                 f"{hist[-1]['psnr']:.2f} ({time.time() - t0:.0f}s)")
        target = arms["plain"][-1]["psnr"]
        results.append({
            "case": 4100 + i, "plain_final_psnr": target,
            "offset_final_psnr": arms["offset"][-1]["psnr"],
            "warm_final_psnr": arms["warm"][-1]["psnr"],
            "plain_init_psnr": arms["plain"][0]["psnr"],
            "offset_init_psnr": arms["offset"][0]["psnr"],
            "warm_init_psnr": arms["warm"][0]["psnr"],
            "plain_iters_to_target": recon.iters_to_psnr(arms["plain"], target),
            "offset_iters_to_target": recon.iters_to_psnr(arms["offset"], target),
            "warm_iters_to_target": recon.iters_to_psnr(arms["warm"], target),
        })
    summary = {
        "config": dict(n_train=n_train, n_test=n_test, train_vox=train_vox, test_vox=test_vox,
                       g_train=g_train, g_test=g_test, train_iters=train_iters,
                       test_iters=test_iters, net_steps=net_steps, batch=batch, lr=lr),
        "net_loss": losses, "cases": results,
        "constant_offsets": {"log_scale": d_off, "logit": e_off},
        "plain_iters": test_iters, "seconds": time.time() - t0,
    }
    for arm in ("offset", "warm"):
        reached = [r[f"{arm}_iters_to_target"] for r in results
                   if r[f"{arm}_iters_to_target"] is not None]
        summary[f"{arm}_reached"] = f"{len(reached)}/{len(results)}"
        summary[f"{arm}_iters_mean"] = float(np.mean(reached)) if reached else None
        summary[f"{arm}_iters_median"] = float(np.median(reached)) if reached else None
    if out:
        with open(out, "w") as f:
            json.dump(summary, f, indent=1)
    return summary


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=64)
    ap.add_argument("--n-test", type=int, default=16)
    ap.add_argument("--train-vox", type=int, default=128)
    ap.add_argument("--test-vox", type=int, default=256)
    ap.add_argument("--g-train", type=int, default=50)
    ap.add_argument("--g-test", type=int, default=100)
    ap.add_argument("--train-iters", type=int, default=200)
    ap.add_argument("--test-iters", type=int, default=1000)
    ap.add_argument("--net-steps", type=int, default=1500)
    ap.add_argument("--out", default=None)
    ap.add_argument("--md", default=None, help="also write the per-phantom table here")
    a = ap.parse_args()
    s = run_experiment(a.n_train, a.n_test, a.train_vox, a.test_vox, a.g_train, a.g_test,
                       a.train_iters, a.test_iters, a.net_steps, out=a.out)
    print(json.dumps({k: v for k, v in s.items() if k != "cases"}))
    if a.md:
        def it(v):
            return "not reached" if v is None else str(v)
        rows = ["| phantom seed | plain init dB | plain final dB | offset init dB | offset final dB "
                "| offset iterations to target | warm init dB | warm final dB | warm iterations to "
                "target |", "|---|---|---|---|---|---|---|---|---|"]
        for c in s["cases"]:
            rows.append(f"| {c['case']} | {c['plain_init_psnr']:.2f} | {c['plain_final_psnr']:.2f} "
                        f"| {c['offset_init_psnr']:.2f} | {c['offset_final_psnr']:.2f} | "
                        f"{it(c['offset_iters_to_target'])} | {c['warm_init_psnr']:.2f} | "
                        f"{c['warm_final_psnr']:.2f} | {it(c['warm_iters_to_target'])} |")
        with open(a.md, "w") as f:
            f.write("\n".join(rows) + "\n")

"""Warm-start network in FP64 (test infrastructure only).

Per Gaussian i with centre mu_i: a 3-channel patch X0[c][z][y][x] of 8^3 samples, channel c
= stack c sampled trilinearly (zero outside the stack's index domain) at the world points
mu_i + ((x, y, z) - 3.5) * spacing; then
  conv1 3->32 (3^3, stride 1, pad 1) + b, SiLU     8^3
  conv2 32->32 (3^3, stride 2, pad 1) + b, SiLU    4^3
  conv3 32->32 (3^3, stride 2, pad 1) + b, SiLU    2^3
  conv4 32->32 (2^3, valid) + b, SiLU              1
  linear 32->8 + b  ->  (ds 3, dq 4, dlogit 1)
and the initial parameters are s = s0 + ds, q = (1,0,0,0) + dq, logit = logit0 + dlogit
(residuals on top of the devoxelization initialisation).

Training loss per Gaussian (a covariance-space reading, since (s, q) is not unique: axis
permutations and q ~ -q give the same Gaussian):
  ||Sigma(s, q) - Sigma*||_F^2 / ||Sigma*||_F^2 + (logit - logit*)^2, averaged.
Conv weights are [out][in][kz][ky][kx] flattened; the BF16-valued weights the GPU uses are
exact in FP64.
"""
from __future__ import annotations

import numpy as np

from . import gauss

LAYERS = [  # (c_in, c_out, k, stride, pad, d_in, d_out)
    (3, 32, 3, 1, 1, 8, 8),
    (32, 32, 3, 2, 1, 8, 4),
    (32, 32, 3, 2, 1, 4, 2),
    (32, 32, 2, 1, 0, 2, 1),
]


def trilinear_zero(vol, p):
    """Trilinear value of vol[z,y,x] at index point p, 0 unless p lies in [0, n-1]^3."""
    nz, ny, nx = vol.shape
    if not (0 <= p[0] <= nx - 1 and 0 <= p[1] <= ny - 1 and 0 <= p[2] <= nz - 1):
        return 0.0
    return gauss._trilinear_index(vol, p)


def gather(stacks, stack_data, means, spacing):
    """Patches [B, 3, 8, 8, 8] (FP64)."""
    B = means.shape[0]
    X = np.zeros((B, len(stacks), 8, 8, 8))
    offs = (np.arange(8) - 3.5) * spacing
    for i in range(B):
        for k, (grid, data) in enumerate(zip(stacks, stack_data)):
            A = np.asarray(grid.world_to_index, np.float64)
            for z in range(8):
                for y in range(8):
                    for x in range(8):
                        w = np.asarray(means[i], np.float64) + np.array([offs[x], offs[y], offs[z]])
                        p = A[:, :3] @ w + A[:, 3]
                        X[i, k, z, y, x] = trilinear_zero(data, p)
    return X


def conv3d(X, W, b, k, stride, pad, d_out):
    """X [B, C, D, D, D], W [O, C, k, k, k] -> [B, O, d_out^3] (plain loops over taps)."""
    B, C, D = X.shape[0], X.shape[1], X.shape[2]
    Xp = np.zeros((B, C, D + 2 * pad, D + 2 * pad, D + 2 * pad))
    Xp[:, :, pad:pad + D, pad:pad + D, pad:pad + D] = X
    Z = np.zeros((B, W.shape[0], d_out, d_out, d_out))
    for kz in range(k):
        for ky in range(k):
            for kx in range(k):
                sl = Xp[:, :, kz:kz + stride * d_out:stride, ky:ky + stride * d_out:stride,
                        kx:kx + stride * d_out:stride]
                Z += np.einsum("bczyx,oc->bozyx", sl, W[:, :, kz, ky, kx])
    return Z + b[None, :, None, None, None]


def forward(net, X0):
    """net: dict W1..W4 ([O, C, k, k, k]), b1..b4, Wl [8, 32], bl [8].  Returns (out [B, 8],
    cache)."""
    a = X0
    cache = []
    for l, (ci, co, k, st, pd, di, do) in enumerate(LAYERS):
        z = conv3d(a, net[f"W{l + 1}"], net[f"b{l + 1}"], k, st, pd, do)
        cache.append((a, z))
        a = gauss_silu(z)
    a4 = a.reshape(a.shape[0], 32)
    out = a4 @ net["Wl"].T + net["bl"]
    return out, cache, a4


def gauss_silu(z):
    return z / (1.0 + np.exp(-z))


def assemble(out, s0, logit0):
    s = s0 + out[:, 0:3]
    q = out[:, 3:7] + np.array([1.0, 0.0, 0.0, 0.0])
    logit = logit0 + out[:, 7]
    return s, q, logit


def covariance(s, q):
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    R = gauss.quat_to_rot(qn)
    return np.einsum("nij,nj,nkj->nik", R, np.exp(2 * s), R)


def loss(out, s0, logit0, sig_t, logit_t):
    s, q, lg = assemble(out, s0, logit0)
    S = covariance(s, q)
    num = ((S - sig_t) ** 2).sum((1, 2))
    den = (sig_t ** 2).sum((1, 2))
    return float(np.mean(num / den + (lg - logit_t) ** 2))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def loss_grad(out, s0, logit0, sig_t, logit_t):
    """Loss and dL/d(out) [B, 8] (FP64): dL/dSigma = 2 (Sigma - Sigma*) / (|Sigma*|^2 B), then
    Sigma = R diag(e^{2s}) R^T, R(q/|q|) as in the rendering chain."""
    B = out.shape[0]
    s, q, lg = assemble(out, s0, logit0)
    qnorm = np.linalg.norm(q, axis=1)
    qn = q / qnorm[:, None]
    R = gauss.quat_to_rot(qn)
    S2 = np.exp(2 * s)
    S = np.einsum("nij,nj,nkj->nik", R, S2, R)
    den = (sig_t ** 2).sum((1, 2))
    L = float(np.mean(((S - sig_t) ** 2).sum((1, 2)) / den + (lg - logit_t) ** 2))
    G = 2 * (S - sig_t) / (den * B)[:, None, None]
    GR = 2 * np.einsum("nij,njk,nk->nik", G, R, S2)
    RtGR = np.einsum("nji,njk,nkl->nil", R, G, R)
    ds = 2 * S2 * np.einsum("nii->ni", RtGR)
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    g = GR
    dqn = np.stack([
        2 * (-z * g[:, 0, 1] + y * g[:, 0, 2] + z * g[:, 1, 0] - x * g[:, 1, 2] - y * g[:, 2, 0] + x * g[:, 2, 1]),
        2 * (y * g[:, 0, 1] + z * g[:, 0, 2] + y * g[:, 1, 0] - 2 * x * g[:, 1, 1] - w * g[:, 1, 2]
             + z * g[:, 2, 0] + w * g[:, 2, 1] - 2 * x * g[:, 2, 2]),
        2 * (-2 * y * g[:, 0, 0] + x * g[:, 0, 1] + w * g[:, 0, 2] + x * g[:, 1, 0] + z * g[:, 1, 2]
             - w * g[:, 2, 0] + z * g[:, 2, 1] - 2 * y * g[:, 2, 2]),
        2 * (-2 * z * g[:, 0, 0] - w * g[:, 0, 1] + x * g[:, 0, 2] + w * g[:, 1, 0] - 2 * z * g[:, 1, 1]
             + y * g[:, 1, 2] + x * g[:, 2, 0] + y * g[:, 2, 1]),
    ], axis=1)
    dq = (dqn - qn * (qn * dqn).sum(1, keepdims=True)) / qnorm[:, None]
    dlg = 2 * (lg - logit_t) / B
    return L, np.concatenate([ds, dq, dlg[:, None]], axis=1)


def conv3d_backward(X, W, dZ, k, stride, pad):
    """Gradients of a conv3d layer: (dX [B, C, D^3], dW [O, C, k^3], db [O])."""
    B, C, D = X.shape[0], X.shape[1], X.shape[2]
    do = dZ.shape[2]
    Xp = np.zeros((B, C, D + 2 * pad, D + 2 * pad, D + 2 * pad))
    Xp[:, :, pad:pad + D, pad:pad + D, pad:pad + D] = X
    dXp = np.zeros_like(Xp)
    dW = np.zeros_like(W)
    for kz in range(k):
        for ky in range(k):
            for kx in range(k):
                idx = (slice(None), slice(None), slice(kz, kz + stride * do, stride),
                       slice(ky, ky + stride * do, stride), slice(kx, kx + stride * do, stride))
                dW[:, :, kz, ky, kx] = np.einsum("bozyx,bczyx->oc", dZ, Xp[idx])
                dXp[idx] += np.einsum("bozyx,oc->bczyx", dZ, W[:, :, kz, ky, kx])
    return dXp[:, :, pad:pad + D, pad:pad + D, pad:pad + D], dW, dZ.sum((0, 2, 3, 4))


def backward(net, X0, dout):
    """Weight gradients of sum(out * dout) (FP64)."""
    out, cache, a4 = forward(net, X0)
    g = {"Wl": dout.T @ a4, "bl": dout.sum(0)}
    da = (dout @ net["Wl"]).reshape(-1, 32, 1, 1, 1)
    for l in range(len(LAYERS) - 1, -1, -1):
        ci, co, k, st, pd, di, do = LAYERS[l]
        a_in, z = cache[l]
        dz = da * dsilu(z)
        dX, g[f"W{l + 1}"], g[f"b{l + 1}"] = conv3d_backward(a_in, net[f"W{l + 1}"], dz, k, st, pd)
        da = dX
    return g

"""Neural residual field (paper Sec. 3.4, Eq. 8) in FP64.  Test infrastructure only.

r(x) = out_scale * tanh(w_out . a_D + b_out), a_l = SiLU(W_l a_{l-1} + b_l) for l = 1..D,
a_0 = gamma(x) = (x, sin(2^k pi x), cos(2^k pi x) for k = 0..L-1) — the NeRF-style Fourier
encoding with the input kept, features ordered [x(3), then per band k: sin(3), cos(3)],
zero-padded to in_pad.  Weights are the BF16-valued weights the GPU uses, exact in FP64.

World coordinates of voxel v on a grid are x = float32(((M00 vx + M01 vy) + M02 vz) + M03)
per row of the index->world affine M, evaluated in binary64 without contraction and rounded
once to float32 (the GPU follows the same recipe, so both sides encode the same x; the
high bands make the encoding extremely sensitive to x).  The phase of band k is the exact
float scaling phi = x 2^{k-1}; frac = phi - rint(phi) (exact); the features are
sin(2 pi frac), cos(2 pi frac).
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """float32 -> bfloat16 (round to nearest even), returned as float32 values."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def bf16_bits(a):
    return (bf16_round(a).view(np.uint32) >> 16).astype(np.uint16)


def index_to_world(world_to_index):
    """Inverse of a grid's world->index affine A = [L | t] (row-major 3x4, binary64) by the
    adjugate: with cofactors c00 = e j - f i, c01 = f h - d j, c02 = d i - e h of
    L = [[a b c] [d e f] [h i j]] and det = a c00 + b c01 + c c02, L^-1 row by row =
    [c00, c i - b j, b f - c e] / det, [c01, a j - c h, c d - a f] / det,
    [c02, b h - a i, a e - b d] / det; the translation column is -(L^-1 t), each row summed in
    column order.  Every product and sum is one binary64 operation in the written order (the
    residual field's coordinates depend on the last bit of this matrix, so the boundary fixes
    the recipe)."""
    A = np.asarray(world_to_index, np.float64).reshape(3, 4)
    a, b, c = float(A[0, 0]), float(A[0, 1]), float(A[0, 2])
    d, e, f = float(A[1, 0]), float(A[1, 1]), float(A[1, 2])
    h, i, j = float(A[2, 0]), float(A[2, 1]), float(A[2, 2])
    c00, c01, c02 = e * j - f * i, f * h - d * j, d * i - e * h
    det = a * c00 + b * c01 + c * c02
    Li = [[c00 / det, (c * i - b * j) / det, (b * f - c * e) / det],
          [c01 / det, (a * j - c * h) / det, (c * d - a * f) / det],
          [c02 / det, (b * h - a * i) / det, (a * e - b * d) / det]]
    M = np.zeros((3, 4))
    for r in range(3):
        M[r, :3] = Li[r]
        M[r, 3] = -((Li[r][0] * float(A[0, 3]) + Li[r][1] * float(A[1, 3])) + Li[r][2] * float(A[2, 3]))
    return M


def world_coords(vox, index_to_world):
    """vox [P,3] integer (x, y, z) -> float32 world coordinates by the stated recipe."""
    M = np.asarray(index_to_world, np.float64).reshape(3, 4)
    v = np.asarray(vox, np.float64)
    out = np.empty(v.shape, np.float32)
    for a in range(3):
        out[:, a] = (((M[a, 0] * v[:, 0] + M[a, 1] * v[:, 1]) + M[a, 2] * v[:, 2]) + M[a, 3])
    return out


def encode(x32, n_freq, in_pad):
    """Fourier features [P, in_pad] (float64) of float32 coordinates."""
    x = np.asarray(x32, np.float32).astype(np.float64)
    P = x.shape[0]
    f = np.zeros((P, in_pad))
    f[:, 0:3] = x
    for k in range(n_freq):
        phi = x * 2.0 ** (k - 1)
        frac = phi - np.rint(phi)
        f[:, 3 + 6 * k: 6 + 6 * k] = np.sin(2 * np.pi * frac)
        f[:, 6 + 6 * k: 9 + 6 * k] = np.cos(2 * np.pi * frac)
    return f


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(weights, feats, out_scale=0.1):
    """weights: dict W (list of [out,in] arrays, first [width, in_pad]), b (list), w_out
    [width], b_out (scalar).  Returns r [P] and the per-layer (z, a) for the backward."""
    a = feats
    zs, acts = [], [a]
    for W, b in zip(weights["W"], weights["b"]):
        z = a @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        a = silu(z)
        zs.append(z)
        acts.append(a)
    zo = a @ np.asarray(weights["w_out"], np.float64) + float(weights["b_out"])
    return out_scale * np.tanh(zo), zs, acts, zo


def backward(weights, feats, dl_dr, out_scale=0.1):
    """Gradients of sum_p dl_dr[p] r(x_p) with respect to every weight (FP64)."""
    r, zs, acts, zo = forward(weights, feats, out_scale)
    dzo = np.asarray(dl_dr, np.float64) * out_scale * (1.0 - np.tanh(zo) ** 2)
    g = {"w_out": acts[-1].T @ dzo, "b_out": dzo.sum(), "W": [None] * len(zs), "b": [None] * len(zs)}
    da = np.outer(dzo, np.asarray(weights["w_out"], np.float64))
    for l in range(len(zs) - 1, -1, -1):
        dz = da * dsilu(zs[l])
        g["W"][l] = dz.T @ acts[l]
        g["b"][l] = dz.sum(0)
        da = dz @ np.asarray(weights["W"][l], np.float64)
    return g

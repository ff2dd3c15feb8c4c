"""Resolution transition of multi-resolution progressive training (Sec. 4.1.3), FP64.

Test infrastructure only (see the package docstring).

The Gaussians of a G^3 lattice (Gaussian (ix, iy, iz) at index (iz G + iy) G + ix, centred on
cell (ix, iy, iz) of [-1, 1]^3 at initialisation) are replaced, at a milestone, by those of a
G'^3 lattice whose parameters are interpolated from the previous lattice: trilinearly for
intensity and scale, by normalised linear interpolation for the rotation quaternions.  The
paper says no more; readings taken:
  - the new Gaussians sit at the new lattice's cell centres c' = -1 + (2 i + 1) / G';
  - the old lattice is sampled at c' in its own cell-index coordinates u = (c' + 1) G / 2 - 1/2,
    clamped to [0, G - 1], with the usual 8-corner trilinear weights;
  - intensity = alpha = sigmoid(logit) is interpolated (a convex combination stays in [0, 1]),
    then clipped to [1e-6, 1 - 1e-6] and mapped back to a logit;
  - scale = exp(log_scale) is interpolated per axis, then multiplied by G / G' (the ratio of the
    lattice spacings), so that every Gaussian keeps covering one lattice cell as at
    initialisation (sigma = h / 2) and the rendered intensity is preserved;
  - each quaternion is normalised, the eight are brought into the hemisphere of the one with
    the largest weight (q and -q are the same rotation), and the weighted sum is normalised
    (the identity if it vanishes).
"""
from __future__ import annotations

import numpy as np


def _corners(u, n):
    """Trilinear corner indices and weights along one axis for continuous indices u."""
    u = np.clip(u, 0.0, n - 1.0)
    i0 = np.minimum(np.floor(u).astype(np.int64), max(n - 2, 0))
    f = u - i0
    i1 = np.minimum(i0 + 1, n - 1)
    return (i0, i1), (1.0 - f, f)


def upsample(quat, log_scale, logit, g_old, g_new):
    """New lattice (mean, quat, log_scale, logit) [g_new^3, ...] from the old lattice's."""
    q = np.asarray(quat, np.float64).reshape(g_old, g_old, g_old, 4)
    s = np.exp(np.asarray(log_scale, np.float64)).reshape(g_old, g_old, g_old, 3)
    a = 1.0 / (1.0 + np.exp(-np.asarray(logit, np.float64))).reshape(g_old, g_old, g_old)
    qn = q / np.linalg.norm(q, axis=-1, keepdims=True)
    c = -1.0 + (2.0 * np.arange(g_new) + 1.0) / g_new          # new cell centres
    u = (c + 1.0) * g_old / 2.0 - 0.5                          # in old cell-index units
    (i0, i1), (w0, w1) = _corners(u, g_old)
    n = g_new ** 3
    mean = np.zeros((n, 3))
    out_q = np.zeros((n, 4))
    out_s = np.zeros((n, 3))
    out_a = np.zeros(n)
    idx = 0
    for iz in range(g_new):
        for iy in range(g_new):
            for ix in range(g_new):
                corners = []
                for dz in (0, 1):
                    for dy in (0, 1):
                        for dx in (0, 1):
                            z = (i0, i1)[dz][iz]
                            y = (i0, i1)[dy][iy]
                            x = (i0, i1)[dx][ix]
                            w = (w0, w1)[dz][iz] * (w0, w1)[dy][iy] * (w0, w1)[dx][ix]
                            corners.append((w, z, y, x))
                wa = sum(w * a[z, y, x] for w, z, y, x in corners)
                ws = sum(w * s[z, y, x] for w, z, y, x in corners)
                ref = max(range(8), key=lambda k: (corners[k][0], -k))
                qr = qn[corners[ref][1], corners[ref][2], corners[ref][3]]
                qs = np.zeros(4)
                for w, z, y, x in corners:
                    qk = qn[z, y, x]
                    qs = qs + w * (qk if np.dot(qk, qr) >= 0 else -qk)
                nq = np.linalg.norm(qs)
                out_q[idx] = qs / nq if nq > 0 else np.array([1.0, 0.0, 0.0, 0.0])
                out_s[idx] = ws * (g_old / g_new)
                out_a[idx] = min(max(wa, 1e-6), 1.0 - 1e-6)
                mean[idx] = (c[ix], c[iy], c[iz])
                idx += 1
    return mean, out_q, np.log(out_s), np.log(out_a / (1.0 - out_a))

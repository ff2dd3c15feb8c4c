"""SSIM term of the reconstruction loss (Sec. 3.5.2, Eq. 10) on whole stack slices, FP64.

Test infrastructure only (see the package docstring).

The paper adds lambda_SSIM L_SSIM to the smooth-L1 data term (Eq. 10, lambda_SSIM = 0.5 in
Sec. 4.1.4) and notes that SSIM needs whole slices; it gives neither the window nor the
constants.  Reading taken: every z-slice of a stack is a 2D image, compared with the textbook
SSIM of Wang et al. (2004):
  - an 11 x 11 Gaussian window of standard deviation 1.5, normalised to sum 1;
  - stabilising constants C1 = (0.01 D)^2, C2 = (0.03 D)^2 with dynamic range D = 1 (the
    intensities are normalised to [0, 1], Sec. 3.1);
  - local statistics over the window with zero padding outside the slice, so that the SSIM
    map has the slice's size;
  - L_SSIM = 1 - the mean of the map over every pixel of every slice of every stack (the
    same voxel set the smooth-L1 mean runs over).

For pixel p with local means mu_x, mu_y, local second moments m_xx, m_yy, m_xy (window sums of
x^2, y^2, x y), sigma_x^2 = m_xx - mu_x^2, sigma_y^2 = m_yy - mu_y^2, sigma_xy = m_xy - mu_x mu_y:
    S(p) = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)).

Gradient with respect to the prediction x: each window sum is linear in x, so
    dS(p)/dx_q = w(q - p) [dS/dmu_x + 2 x_q dS/dm_xx + y_q dS/dm_xy](p),
with (mu_x, m_xx, m_xy) taken as the independent variables; summing over p is the adjoint of
the window sum.  Every function runs in float64, or complex128 for complex-step checks.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

WIN = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window(size: int = WIN, sigma: float = SIGMA) -> np.ndarray:
    """1D Gaussian taps g[k] proportional to exp(-(k - size//2)^2 / (2 sigma^2)), sum 1; the
    2D window is the outer product g g^T."""
    k = np.arange(size, dtype=np.float64) - size // 2
    g = np.exp(-k * k / (2.0 * sigma * sigma))
    return g / g.sum()


def window_sum(img: np.ndarray, w2: np.ndarray) -> np.ndarray:
    """out[p] = sum_{i,j} w2[i, j] img[p_y + i - r, p_x + j - r], zero outside the image
    (r = half width).  img [ny, nx]."""
    ny, nx = img.shape
    r = w2.shape[0] // 2
    pad = np.zeros((ny + 2 * r, nx + 2 * r), dtype=img.dtype)
    pad[r:r + ny, r:r + nx] = img
    out = np.zeros_like(img)
    for i in range(2 * r + 1):
        for j in range(2 * r + 1):
            out = out + w2[i, j] * pad[i:i + ny, j:j + nx]
    return out


def window_sum_adjoint(v: np.ndarray, w2: np.ndarray) -> np.ndarray:
    """Adjoint of window_sum: out[q] = sum_p w2[q_y - p_y + r, q_x - p_x + r] v[p] over the
    map positions p inside the image."""
    ny, nx = v.shape
    r = w2.shape[0] // 2
    pad = np.zeros((ny + 2 * r, nx + 2 * r), dtype=v.dtype)
    pad[r:r + ny, r:r + nx] = v
    out = np.zeros_like(v)
    for i in range(2 * r + 1):
        for j in range(2 * r + 1):
            # p = q - (i - r, j - r)
            out = out + w2[i, j] * pad[2 * r - i:2 * r - i + ny, 2 * r - j:2 * r - j + nx]
    return out


def _stats(x, y, w2):
    mx, my = window_sum(x, w2), window_sum(y, w2)
    mxx, myy, mxy = window_sum(x * x, w2), window_sum(y * y, w2), window_sum(x * y, w2)
    return mx, my, mxx, myy, mxy


def ssim_map(x: np.ndarray, y: np.ndarray, w2: np.ndarray | None = None) -> np.ndarray:
    """SSIM map of one 2D slice pair (float64 or complex128)."""
    if w2 is None:
        g = window()
        w2 = np.outer(g, g)
    x = _as(x)
    y = _as(y)
    mx, my, mxx, myy, mxy = _stats(x, y, w2)
    vx, vy, cxy = mxx - mx * mx, myy - my * my, mxy - mx * my
    return ((2 * mx * my + C1) * (2 * cxy + C2)) / ((mx * mx + my * my + C1) * (vx + vy + C2))


def _as(a):
    a = np.asarray(a)
    return a if np.iscomplexobj(a) else a.astype(np.float64)


def ssim_slice(x: np.ndarray, y: np.ndarray):
    """One slice pair: (sum of its SSIM map, d(sum of the map)/dx)."""
    g = window()
    w2 = np.outer(g, g)
    x, y = _as(x), _as(y)
    mx, my, mxx, myy, mxy = _stats(x, y, w2)
    vx, vy, cxy = mxx - mx * mx, myy - my * my, mxy - mx * my
    a1, a2 = 2 * mx * my + C1, 2 * cxy + C2
    b1, b2 = mx * mx + my * my + C1, vx + vy + C2
    s = (a1 * a2) / (b1 * b2)
    # partial derivatives of S with (mu_x, m_xx, m_xy) independent
    d_mx = (2 * my * a2 - 2 * my * a1) / (b1 * b2) - 2 * mx * s / b1 + 2 * mx * s / b2
    d_mxx = -s / b2
    d_mxy = 2 * a1 / (b1 * b2)
    grad = (window_sum_adjoint(d_mx, w2) + 2 * x * window_sum_adjoint(d_mxx, w2)
            + y * window_sum_adjoint(d_mxy, w2))
    return s.sum(), grad


def ssim_loss(preds: Sequence[np.ndarray], targets: Sequence[np.ndarray]):
    """L_SSIM = 1 - mean SSIM over every slice of every stack ([nz, ny, nx] arrays), and its
    gradient with respect to each prediction.  Returns (value, [grad per stack])."""
    ntot = sum(np.asarray(p).size for p in preds)
    total = 0.0
    grads = []
    for p, t in zip(preds, targets):
        x3, y3 = _as(p), _as(t)
        gr = np.zeros_like(x3)
        for z in range(x3.shape[0]):
            ssum, sgrad = ssim_slice(x3[z], y3[z])
            total = total + ssum
            gr[z] = -sgrad / ntot
        grads.append(gr)
    return 1.0 - total / ntot, grads

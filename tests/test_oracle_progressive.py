"""Pins of the resolution transition of progressive training (Sec. 4.1.3): scipy's trilinear
interpolator, the same-resolution identity, linear fields, quaternion sign invariance, and
preservation of the rendered intensity."""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from oracle import gauss
from oracle import progressive as P
from paper_2603_00145_amd import inputs


def lattice(g, rng, iso=False):
    c = -1.0 + (2.0 * np.arange(g) + 1.0) / g
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    n = g ** 3
    q = rng.normal(size=(n, 4))
    ls = np.full((n, 3), np.log(1.0 / g)) if iso else np.log(1.0 / g) + rng.normal(0, 0.2, (n, 3))
    logit = rng.normal(0, 1, n)
    mean = np.stack([X, Y, Z], -1).reshape(-1, 3)
    return mean, q, ls, logit


def test_trilinear_matches_scipy():
    rng = np.random.default_rng(0)
    g0, g1 = 5, 8
    _, q, ls, logit = lattice(g0, rng)
    mean, _, ls1, logit1 = P.upsample(q, ls, logit, g0, g1)
    idx = np.arange(g0, dtype=np.float64)
    a = 1 / (1 + np.exp(-logit.reshape(g0, g0, g0)))
    s = np.exp(ls.reshape(g0, g0, g0, 3))
    u = np.clip((mean + 1.0) * g0 / 2.0 - 0.5, 0, g0 - 1)[:, ::-1]    # (z, y, x)
    ra = RegularGridInterpolator((idx, idx, idx), a)(u)
    np.testing.assert_allclose(1 / (1 + np.exp(-logit1)), ra, rtol=1e-12)
    for m in range(3):
        rs = RegularGridInterpolator((idx, idx, idx), s[..., m])(u) * g0 / g1
        np.testing.assert_allclose(np.exp(ls1[:, m]), rs, rtol=1e-12)


def test_same_resolution_is_identity():
    rng = np.random.default_rng(1)
    g = 4
    mean, q, ls, logit = lattice(g, rng)
    m1, q1, ls1, lg1 = P.upsample(q, ls, logit, g, g)
    np.testing.assert_allclose(m1, mean, atol=1e-15)
    np.testing.assert_allclose(ls1, ls, atol=1e-12)
    np.testing.assert_allclose(lg1, logit, atol=1e-9)
    np.testing.assert_allclose(q1, q / np.linalg.norm(q, axis=1, keepdims=True), atol=1e-15)


def test_linear_alpha_field_reproduced():
    rng = np.random.default_rng(2)
    g0, g1 = 6, 10
    mean, q, ls, _ = lattice(g0, rng)
    alpha = 0.5 + 0.2 * mean[:, 0] - 0.1 * mean[:, 1] + 0.15 * mean[:, 2]
    m1, _, _, lg1 = P.upsample(q, ls, np.log(alpha / (1 - alpha)), g0, g1)
    inner = np.all(np.abs(m1) <= 1.0 - 1.0 / g0, axis=1)     # inside the old centres' hull
    ref = 0.5 + 0.2 * m1[:, 0] - 0.1 * m1[:, 1] + 0.15 * m1[:, 2]
    np.testing.assert_allclose((1 / (1 + np.exp(-lg1)))[inner], ref[inner], rtol=1e-12)


def test_quaternion_sign_does_not_matter():
    rng = np.random.default_rng(3)
    g0, g1 = 3, 5
    _, _, ls, logit = lattice(g0, rng)
    q0 = np.array([0.8, 0.1, -0.5, 0.3])
    signs = rng.choice([-1.0, 1.0], size=g0 ** 3)
    q = signs[:, None] * q0[None] * rng.uniform(0.5, 2.0, size=(g0 ** 3, 1))
    _, q1, _, _ = P.upsample(q, ls, logit, g0, g1)
    np.testing.assert_allclose(np.abs(q1 @ (q0 / np.linalg.norm(q0))), 1.0, atol=1e-14)


def test_rendered_intensity_preserved():
    """Isotropic lattices with sigma = h/2 and a smooth alpha: the volume rendered from the
    refined lattice matches the coarse one's in the interior (mean within 1%, every voxel
    within the lattice ripple)."""
    rng = np.random.default_rng(4)
    g0, g1, n = 8, 12, 24
    mean, q, ls, _ = lattice(g0, rng, iso=True)
    ls = ls + np.log(0.5 * 2.0)          # sigma = h/2 with h = 2/g
    alpha = 0.3 + 0.2 * np.cos(1.5 * mean[:, 0]) * np.cos(mean[:, 1])
    vol = inputs.volume_grid(n)

    def render(mean, q, ls, logit):
        g = inputs.Gaussians(mean.astype(np.float32), q.astype(np.float32),
                             ls.astype(np.float32), logit.astype(np.float32))
        (gt, lo, hi, ne, _), = gauss.prepare(g, [vol])
        return gauss.render(vol, gt, lo, hi, ne)
    coarse = render(mean, q, ls, np.log(alpha / (1 - alpha)))
    m1, q1, ls1, lg1 = P.upsample(q, ls, np.log(alpha / (1 - alpha)), g0, g1)
    fine = render(m1, q1, ls1, lg1)
    inner = (slice(6, -6),) * 3
    # the lattice sums ripple by a few percent (sigma = h/2, 3-sigma boxes) at different phases;
    # without the spacing factor the fine lattice would render (12/8)^3 = 3.4x brighter
    mean_rel = abs(fine[inner].mean() - coarse[inner].mean()) / coarse[inner].mean()
    max_rel = np.abs(fine[inner] - coarse[inner]).max() / np.abs(coarse[inner]).max()
    assert mean_rel < 0.01, mean_rel
    assert max_rel < 0.06, max_rel

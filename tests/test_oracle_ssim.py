"""Pins of the SSIM oracle (Eq. 10's L_SSIM, read as textbook SSIM on whole stack slices)
against library routines, closed forms, invariants and complex-step differentiation."""
import numpy as np
import pytest
from scipy import ndimage
from scipy.signal import windows

from oracle import ssim as S


def _w2():
    g = S.window()
    return np.outer(g, g)


def test_window_is_the_library_gaussian():
    ref = windows.gaussian(11, std=1.5)
    np.testing.assert_allclose(S.window(), ref / ref.sum(), rtol=0, atol=1e-16)
    assert abs(S.window().sum() - 1.0) < 1e-15


@pytest.mark.parametrize("shape", [(13, 7), (3, 2), (1, 1), (24, 31)])
def test_window_sum_is_zero_padded_correlation(shape):
    rng = np.random.default_rng(sum(shape))
    img = rng.random(shape)
    w2 = _w2()
    ref = ndimage.correlate(img, w2, mode="constant", cval=0.0)
    np.testing.assert_allclose(S.window_sum(img, w2), ref, rtol=1e-13, atol=1e-15)


def test_window_sum_adjoint_dot_product():
    rng = np.random.default_rng(3)
    w2 = _w2()
    u, v = rng.standard_normal((9, 14)), rng.standard_normal((9, 14))
    lhs = np.sum(S.window_sum(u, w2) * v)
    rhs = np.sum(u * S.window_sum_adjoint(v, w2))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_identical_slices_give_one_and_zero_gradient():
    rng = np.random.default_rng(4)
    x = rng.random((2, 17, 12))
    val, (g,) = S.ssim_loss([x], [x])
    assert abs(val) < 1e-14
    np.testing.assert_allclose(S.ssim_map(x[0], x[0]), 1.0, rtol=0, atol=1e-14)
    assert np.abs(g).max() < 1e-13


def test_constant_slices_interior_closed_form():
    a, b = 0.3, 0.7
    x, y = np.full((25, 27), a), np.full((25, 27), b)
    m = S.ssim_map(x, y)
    ref = (2 * a * b + S.C1) / (a * a + b * b + S.C1)   # zero variances inside
    np.testing.assert_allclose(m[5:-5, 5:-5], ref, rtol=1e-12)
    # next to the border the zero padding lowers the means and adds variance
    assert abs(m[0, 0] - ref) > 1e-3


def test_single_pixel_closed_form():
    # a 1 x 1 slice sees only the window centre: mu = w x, m = w x^2 with w = g[5]^2
    a, b = 0.4, 0.9
    w = S.window()[5] ** 2
    mu_x, mu_y = w * a, w * b
    vx, vy, cxy = w * a * a - mu_x ** 2, w * b * b - mu_y ** 2, w * a * b - mu_x * mu_y
    ref = ((2 * mu_x * mu_y + S.C1) * (2 * cxy + S.C2)) / \
        ((mu_x ** 2 + mu_y ** 2 + S.C1) * (vx + vy + S.C2))
    got = S.ssim_map(np.array([[a]]), np.array([[b]]))[0, 0]
    assert abs(got - ref) < 1e-15


def test_symmetric_in_its_arguments():
    rng = np.random.default_rng(5)
    x, y = rng.random((15, 19)), rng.random((15, 19))
    np.testing.assert_allclose(S.ssim_map(x, y), S.ssim_map(y, x), rtol=1e-13)


def test_gradient_matches_complex_step():
    rng = np.random.default_rng(6)
    preds = [rng.random((2, 9, 12)), rng.random((1, 4, 3))]
    targs = [np.clip(p + 0.1 * rng.standard_normal(p.shape), 0, 1) for p in preds]
    _, grads = S.ssim_loss(preds, targs)
    h = 1e-30
    for k, p in enumerate(preds):
        for idx in np.ndindex(p.shape):
            pc = [q.astype(np.complex128) for q in preds]
            pc[k][idx] += 1j * h
            val, _ = S.ssim_loss(pc, targs)
            d = np.imag(val) / h
            assert abs(d - grads[k][idx]) <= 1e-10 * max(1e-3, abs(d)), (k, idx)

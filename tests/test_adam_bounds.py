"""The Adam output ranges used by the training-step GPU tests contain the image of the gradient
interval, checked against dense sampling of that interval (Adam, Sec. 4.1.4)."""
import numpy as np
import pytest

from adam_bounds import adam_range
from oracle import gauss


@pytest.mark.parametrize("t", [1, 2, 7])
def test_range_contains_dense_image(t):
    rng = np.random.default_rng(t)
    n = 1500
    p = rng.normal(size=n)
    m = rng.normal(size=n) * 1e-3
    v = (rng.normal(size=n) * 1e-3) ** 2
    g = rng.normal(size=n) * 1e-3
    delta = np.abs(rng.normal(size=n)) * 1e-3
    lo_hi = adam_range(p, g, delta, m, v, t, 1e-3)
    dense = [gauss.adam(p, g + s * delta, m, v, t, 1e-3) for s in np.linspace(-1, 1, 2001)]
    for (lo, hi), arr in zip(lo_hi, zip(*dense)):
        a = np.stack(arr)
        scale = np.max(np.abs(a)) + 1e-300
        assert np.all(a.min(0) >= lo - 1e-12 * scale)
        assert np.all(a.max(0) <= hi + 1e-12 * scale)

"""Bars for Adam's outputs when the gradient is known only to a bar (shared by the GPU tests of
training steps).

Adam's update divides the first moment by the root of the second, so where the gradient is not
resolved by its bar the update can differ by the order of the learning rate; each output is
therefore required to lie in the image of the gradient bar under the oracle's Adam step,
widened by 1e-5 of the update's (or the moment's) largest magnitude for FP32 arithmetic and by
two float32 spacings of the stored value.

The image of an interval [g - delta, g + delta] is spanned by the outputs at its ends and at the
stationary points inside it: m is linear in g, v is a quadratic with its minimum at g = 0, and
the step m_hat / (sqrt(v_hat) + eps) is not monotone in g once the previous first moment is
non-zero (it peaks where the new gradient slightly exceeds the running mean), so its stationary
points are solved for in closed form below.
"""
import numpy as np

from oracle import gauss

TOL = 1e-5
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def _step_stationary(m, v, t):
    """Roots g of d/dg [(a + b g) / (sqrt(c + d g^2) / sb + eps)] = 0, where m' = a + b g and
    v' = c + d g^2 are Adam's new moments and sb = sqrt(1 - beta2^t).  Setting the derivative
    to zero gives b (c + d g^2) + b eps sb sqrt(c + d g^2) = (a + b g) d g, i.e.
    b eps sb sqrt(c + d g^2) = a d g - b c; squaring leaves a quadratic in g whose real roots
    include every stationary point (a spurious root is still a point of the interval, so it
    cannot widen the image)."""
    a = BETA1 * np.asarray(m, np.float64)
    b = 1.0 - BETA1
    c = BETA2 * np.asarray(v, np.float64)
    d = 1.0 - BETA2
    sb = np.sqrt(1.0 - BETA2 ** t)
    k = (b * EPS * sb) ** 2
    qa = (a * d) ** 2 - k * d
    qb = -2.0 * a * b * c * d
    qc = (b * c) ** 2 - k * c
    disc = qb * qb - 4.0 * qa * qc
    roots = []
    with np.errstate(divide="ignore", invalid="ignore"):
        sq = np.sqrt(np.maximum(disc, 0.0))
        for sgn in (-1.0, 1.0):
            r = (-qb + sgn * sq) / (2.0 * qa)
            roots.append(np.where((disc >= 0) & (qa != 0) & np.isfinite(r), r, np.nan))
    return roots


def adam_range(p, g, delta, m, v, t, lr, k=9):
    """Elementwise range of the oracle's Adam outputs (p, m, v) over g' in [g - delta, g + delta]."""
    g = np.asarray(g, np.float64)
    lo, hi = g - delta, g + delta
    cands = [g + s * delta for s in np.linspace(-1.0, 1.0, k)]
    cands.append(np.clip(np.zeros_like(g), lo, hi))
    for r in _step_stationary(m, v, t):
        cands.append(np.where(np.isnan(r), g, np.clip(r, lo, hi)))
    outs = [gauss.adam(p, gc, m, v, t, lr) for gc in cands]
    return [(np.min(np.stack(x), 0), np.max(np.stack(x), 0)) for x in zip(*outs)]


def check_range(name, got, rng_lo_hi, ref, base):
    lo, hi = rng_lo_hi
    got = np.asarray(got, np.float64)
    scale = np.max(np.abs(ref - base)) if base is not None else np.max(np.abs(ref))
    tol = TOL * scale + 2.0 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    excess = np.maximum(lo - tol - got, got - hi - tol)
    worst = float(np.max(excess)) if excess.size else -1.0
    if worst > 0:
        i = int(np.argmax(excess))
        raise AssertionError(f"{name}: element {i} = {got.reshape(-1)[i]!r} outside "
                             f"[{lo.reshape(-1)[i]!r}, {hi.reshape(-1)[i]!r}] by {worst:.3e} "
                             f"(tol {tol.reshape(-1)[i]:.3e})")
    # how tight: normwise distance to the oracle's own output
    return float(np.max(np.abs(got - ref)) / max(scale, 1e-300)) if got.size else 0.0

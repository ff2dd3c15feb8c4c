"""Bars for Adam's outputs when the gradient is known only to a bar (shared by the GPU tests of
training steps).

Adam's update divides the first moment by the root of the second, so where the gradient is not
resolved by its bar the update can differ by the order of the learning rate; each output is
therefore required to lie in the image of the gradient bar under the oracle's Adam step,
widened by 1e-5 of the update's (or the moment's) largest magnitude for FP32 arithmetic and by
two float32 spacings of the stored value.
"""
import numpy as np

from oracle import gauss

TOL = 1e-5


def adam_range(p, g, delta, m, v, t, lr, k=9):
    """Elementwise range of the oracle's Adam outputs (p, m, v) over g' in [g - delta, g + delta]."""
    outs = [gauss.adam(p, g + s * delta, m, v, t, lr) for s in np.linspace(-1.0, 1.0, k)]
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

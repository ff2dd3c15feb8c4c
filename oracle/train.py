"""One training iteration of the reconstruction in FP64.  Test infrastructure only.

The iteration is the paper's optimisation loop (Sec. 3.5): render every thick-slice stack from
the Gaussians (Eq. 7 with the slice profile, oracle.gauss), add the neural residual field at
each stack voxel when it is on (Sec. 3.4, Eq. 8, oracle.nrf), form the smooth-L1 data term
averaged over every stack voxel (Eq. 11, beta = 1) and its per-voxel gradient, backpropagate to
every raw Gaussian parameter with the anisotropy regulariser added (Eq. 12-13), backpropagate
the same per-voxel gradient into the field's weights, then take one Adam step per parameter
group with the learning rates of Sec. 4.1.4 (PyTorch's arrangement, oracle.gauss.adam).

Inputs are the float32 state an FP32 implementation stores: Gaussian parameters, Adam moments,
the field's float32 master weights and moments.  The field's forward and backward use the BF16
copies of the master weights (round to nearest even of the float32 values), as the kernels do;
every other quantity is binary64.  Boxes come from the float32 parameters by oracle.recipe,
so the set of contributing (Gaussian, voxel) pairs is the one an FP32 implementation bins.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np

from . import gauss
from . import nrf as onrf

GROUPS = ("mean", "quat", "log_scale", "logit")


class _G:
    """Minimal Gaussians container (float32 arrays) for the oracle's box recipe."""

    def __init__(self, mean, quat, log_scale, logit):
        self.mean = np.asarray(mean, np.float32)
        self.quat = np.asarray(quat, np.float32)
        self.log_scale = np.asarray(log_scale, np.float32)
        self.logit = np.asarray(logit, np.float32)

    @property
    def n(self):
        return self.mean.shape[0]


def all_voxels(grid):
    """Integer (x, y, z) of every voxel of a grid, in [nz][ny][nx] memory order."""
    z, y, x = np.meshgrid(np.arange(grid.nz), np.arange(grid.ny), np.arange(grid.nx),
                          indexing="ij")
    return np.stack([x, y, z], -1).reshape(-1, 3)


def field_weights(master: Dict[str, np.ndarray], depth: int):
    """The weights the field's forward uses: matrices and the output vector as the BF16 values
    of the float32 masters, biases as the float32 masters (layout of the kernels' weights:
    w_in [64, in_pad], w_hid [depth-1, 64, 64], b_in [64], b_hid [depth-1, 64], w_out [64],
    b_out [1])."""
    bf = lambda a: onrf.bf16_round(np.asarray(a, np.float32)).astype(np.float64)
    W = [bf(master["w_in"])] + [bf(master["w_hid"][l]) for l in range(depth - 1)]
    b = [np.asarray(master["b_in"], np.float32).astype(np.float64)] + \
        [np.asarray(master["b_hid"][l], np.float32).astype(np.float64) for l in range(depth - 1)]
    return {"W": W, "b": b, "w_out": bf(master["w_out"]),
            "b_out": float(np.asarray(master["b_out"], np.float32).reshape(-1)[0])}


def field_grads_as_master(g, master, depth):
    """Map the oracle's gradient dict (W list, b list, w_out, b_out) onto the masters' layout."""
    out = {k: np.zeros(np.shape(v)) for k, v in master.items()}
    out["w_in"] = np.asarray(g["W"][0])
    out["b_in"] = np.asarray(g["b"][0])
    for l in range(depth - 1):
        out["w_hid"][l] = g["W"][l + 1]
        out["b_hid"][l] = g["b"][l + 1]
    out["w_out"] = np.asarray(g["w_out"])
    out["b_out"] = np.asarray([g["b_out"]]).reshape(np.shape(master["b_out"]))
    return out


def step(params: Sequence[np.ndarray], m: Sequence[np.ndarray], v: Sequence[np.ndarray],
         t: int, stacks, targets: Sequence[np.ndarray], lrs: Sequence[float],
         lam_aniso: float, lam_r: float, field: Optional[dict] = None) -> dict:
    """One iteration from the float32 state (params, m, v of the four groups, Adam step t >= 1).

    field (optional): {"master": dict of float32 arrays, "m": dict, "v": dict, "t": int,
    "lr": float, "n_freq", "in_pad", "depth", "out_scale"}.

    Returns renders (with the field added), the data term (smooth-L1; the anisotropy term
    enters the gradients only), dL/dI per stack, raw gradients of the
    four groups, their new (p, m, v) in binary64, and for the field its weights' gradients and
    new (master, m, v)."""
    g = _G(*params)
    prep = gauss.prepare(g, stacks)
    # the plain sums, each Gaussian visiting its box (identical to the brute force; full size)
    renders = [gauss.render_scatter(gr, gt, lo, hi, ne)
               for gr, (gt, lo, hi, ne, _) in zip(stacks, prep)]
    feats = None
    r_vals = None
    if field is not None:
        W = field_weights(field["master"], field["depth"])
        feats, r_vals = [], []
        for gr in stacks:
            x = onrf.world_coords(all_voxels(gr), onrf.index_to_world(gr.world_to_index))
            f = onrf.encode(x, field["n_freq"], field["in_pad"])
            r, *_ = onrf.forward(W, f, field["out_scale"])
            feats.append(f)
            r_vals.append(r.reshape(gr.shape))
        renders = [I + r for I, r in zip(renders, r_vals)]
    loss, dl = gauss.smooth_l1(renders, targets)
    p64 = gauss.params64(g)
    parts = [gauss.grid_partials(gr, gt, lo, hi, ne, d)
             for gr, (gt, lo, hi, ne, _), d in zip(stacks, prep, dl)]
    d_mu, d_q, d_s, d_a = gauss.chain(*p64, stacks, parts)
    if lam_aniso:
        d_s = d_s + lam_aniso * gauss.aniso(g.log_scale, lam_r)[1]
    grads = (d_mu, d_q, d_s, d_a)
    new_p, new_m, new_v = [], [], []
    for k in range(4):
        p1, m1, v1 = gauss.adam(np.asarray(params[k], np.float32).astype(np.float64), grads[k],
                                m[k], v[k], t, lrs[k])
        new_p.append(p1)
        new_m.append(m1)
        new_v.append(v1)
    out = {"renders": renders, "loss": loss, "dl": dl, "grads": grads, "p": new_p, "m": new_m,
           "v": new_v, "r": r_vals}
    if field is not None:
        W = field_weights(field["master"], field["depth"])
        gsum = None
        for f, d in zip(feats, dl):
            gk = onrf.backward(W, f, d.reshape(-1), field["out_scale"])
            gsum = gk if gsum is None else {
                "W": [a + b for a, b in zip(gsum["W"], gk["W"])],
                "b": [a + b for a, b in zip(gsum["b"], gk["b"])],
                "w_out": gsum["w_out"] + gk["w_out"], "b_out": gsum["b_out"] + gk["b_out"]}
        fg = field_grads_as_master(gsum, field["master"], field["depth"])
        fp, fm, fv = {}, {}, {}
        for k, w0 in field["master"].items():
            fp[k], fm[k], fv[k] = gauss.adam(np.asarray(w0, np.float32).astype(np.float64),
                                             fg[k], field["m"][k], field["v"][k], field["t"],
                                             field["lr"])
        out["field_grads"] = fg
        out["field"] = (fp, fm, fv)
    return out

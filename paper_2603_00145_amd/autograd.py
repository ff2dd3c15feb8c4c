"""torch.autograd.Function over the C ABI: forward = gm_bin + gm_render_stacks, backward =
gm_backward (recomputes each Gaussian's values; no per-voxel contributions are saved).

The bins (records, tile lists, grid-frame partials) are shared, mutable device state: a later
forward on the same Bins overwrites them.  Each forward saves the bins' generation; a backward
that finds it changed bins the saved parameters again before differentiating, so the gradient
is always the one of the parameters its forward rendered.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import api


class GMRender(torch.autograd.Function):
    """Render the Gaussians (mean, quat, log_scale, logit) onto bins.grids[ids]."""

    @staticmethod
    def forward(ctx, mean, quat, log_scale, logit, bins: api.Bins, ids: Sequence[int]):
        p = api.GaussParams(mean.detach().contiguous(), quat.detach().contiguous(),
                            log_scale.detach().contiguous(), logit.detach().contiguous())
        bins.bin(p)
        outs = api.render(bins, list(ids))
        ctx.bins = bins
        ctx.generation = bins.generation
        ctx.grids = list(bins.grids)
        ctx.ids = list(ids)
        ctx.save_for_backward(p.mean, p.quat, p.log_scale, p.logit)
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grad_outs):
        mean, quat, log_scale, logit = ctx.saved_tensors
        p = api.GaussParams(mean, quat, log_scale, logit)
        if ctx.bins.generation != ctx.generation:
            # another forward (or a pose change) re-binned these bins since this forward
            if any(g is not h for g, h in zip(ctx.bins.grids, ctx.grids)):
                ctx.bins.set_grids(ctx.grids)
            ctx.bins.bin(p)
        grads = api.GaussParams.zeros_like(p)
        dl = [(g if g is not None else torch.zeros(ctx.bins.grids[i].shape, device=mean.device))
              .contiguous().to(torch.float32) for g, i in zip(grad_outs, ctx.ids)]
        api.backward(p, ctx.bins, ctx.ids, dl, grads)
        return grads.mean, grads.quat, grads.log_scale, grads.logit, None, None


def render(params: Sequence[torch.Tensor], bins: api.Bins, ids: Sequence[int]):
    """Differentiable rendering: returns one [nz,ny,nx] tensor per listed grid."""
    mean, quat, log_scale, logit = params
    return GMRender.apply(mean, quat, log_scale, logit, bins, tuple(ids))

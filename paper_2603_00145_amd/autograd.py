"""torch.autograd.Function over the C ABI: forward = gm_bin + gm_render_stacks, backward =
gm_backward (recomputes each Gaussian's values; no per-voxel contributions are saved).
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
        ctx.ids = list(ids)
        ctx.save_for_backward(p.mean, p.quat, p.log_scale, p.logit)
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grad_outs):
        mean, quat, log_scale, logit = ctx.saved_tensors
        p = api.GaussParams(mean, quat, log_scale, logit)
        grads = api.GaussParams.zeros_like(p)
        dl = [(g if g is not None else torch.zeros(ctx.bins.grids[i].shape, device=mean.device))
              .contiguous().to(torch.float32) for g, i in zip(grad_outs, ctx.ids)]
        api.backward(p, ctx.bins, ctx.ids, dl, grads)
        return grads.mean, grads.quat, grads.log_scale, grads.logit, None, None


def render(params: Sequence[torch.Tensor], bins: api.Bins, ids: Sequence[int]):
    """Differentiable rendering: returns one [nz,ny,nx] tensor per listed grid."""
    mean, quat, log_scale, logit = params
    return GMRender.apply(mean, quat, log_scale, logit, bins, tuple(ids))

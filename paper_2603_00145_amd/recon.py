"""Reconstruction driver: the paper's training loop (Sec. 3.5; settings of Sec. 4.1.4) run on
the HIP path.  Each iteration bins the Gaussians onto the stacks, renders them, forms the
smooth-L1 data term and its per-voxel gradient (plus, with lambda_ssim > 0, the SSIM term of
Eq. 10 on whole slices), backpropagates to every Gaussian parameter (with the anisotropy
regulariser), and takes one Adam step per parameter group.  Optionally the stacks' rigid
transforms T_k are optimised jointly (Sec. 3.3.2): the library returns the gradient with respect
to each stack's world->index affine and rigid.PoseAdam moves the poses.  With a progressive
schedule (Sec. 4.1.3) the Gaussian lattice is refined at the milestones: the library
interpolates the new lattice from the old one and the optimiser state starts afresh.  Optionally a
neural residual field (Sec. 3.4) is switched on part-way through (delayed activation).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import api, inputs, rigid


@dataclasses.dataclass
class TrainConfig:
    n_iter: int = 200
    lr_mean: float = 1e-3        # position
    lr_quat: float = 1e-3        # rotation
    lr_scale: float = 5e-3       # scale
    lr_logit: float = 5e-2       # intensity
    lambda_aniso: float = 0.1
    lambda_r: float = 1.5
    lambda_ssim: float = 0.0     # 0.5 is the paper's full loss; 0 the plain smooth-L1 method
    psnr_every: int = 10
    nrf: Optional[object] = None  # an nrf.NRF to train jointly (None = Gaussians only)
    nrf_start: float = 0.5        # fraction of n_iter after which the NRF is active
    lr_nrf: float = 1e-4
    nrf_sample: int = 1 << 18     # stack voxels per stack per iteration for the NRF gradient
    optimize_pose: bool = False   # joint optimisation of the stacks' rigid transforms
    pose_mode: str = "stack"      # "stack": one T_k per stack; "slice": one per slice
    lr_pose_rot: float = 1e-3     # radians
    lr_pose_trans: float = 1e-3   # world units ([-1, 1]^3)
    pose_frozen: tuple = (0,)     # stacks whose pose (every slice's, per slice) stays fixed
    block_radius: int = 0         # > 0: the paper's cell-neighbourhood query (Eqs. 4-6)
    cell_resolution: int = 0      # its grid_resolution (cells per axis of [-1, 1]^3)
    lattice: int = 0              # the Gaussians form a lattice^3 (devoxelization layout)
    progressive: tuple = ()       # ((completed iterations, new lattice size), ...) milestones


class Reconstruction:
    """State of one reconstruction: parameters, Adam moments, bins and buffers."""

    def __init__(self, stacks: Sequence, targets: Sequence[torch.Tensor], params: api.GaussParams,
                 cfg: TrainConfig = TrainConfig(), volume_grid=None,
                 phantom: Optional[torch.Tensor] = None,
                 slice_poses: Optional[Sequence] = None):
        self.cfg = cfg
        self.stacks = list(stacks)
        self.targets = [t.contiguous() for t in targets]
        self.p = params
        self.m = api.GaussParams.zeros_like(params)
        self.v = api.GaussParams.zeros_like(params)
        dev = params.mean.device
        self.bins = self._bins(params.n, self.stacks, 10)
        self.ids = list(range(len(self.stacks)))
        self.outs = [torch.empty(s.shape, dtype=torch.float32, device=dev) for s in self.stacks]
        self.dls = [torch.empty(s.shape, dtype=torch.float32, device=dev) for s in self.stacks]
        self.volume_grid = volume_grid
        self.phantom = phantom
        self.vbins = self._bins(params.n, [volume_grid], 12) if volume_grid is not None else None
        self.it = 0
        self.adam_t0 = 0              # Adam's step count restarts at a lattice refinement
        self.nrf_on = False
        self.lattice = cfg.lattice
        if cfg.progressive and self.lattice ** 3 != params.n:
            raise ValueError("a progressive schedule needs the Gaussians of a lattice^3 grid")
        self.poses = None
        self.slices = None
        if cfg.pose_mode not in ("stack", "slice"):
            raise ValueError("pose_mode is 'stack' or 'slice'")
        if cfg.optimize_pose and cfg.pose_mode == "slice":
            self._init_slices(slice_poses)
        elif cfg.optimize_pose:
            self.poses = [rigid.StackPose(s) for s in self.stacks]
            self.pose_opt = rigid.PoseAdam(self.poses, cfg.lr_pose_rot, cfg.lr_pose_trans,
                                           frozen=cfg.pose_frozen)

    # slices per Bins (the library bins at most 8 grids at once)
    SLICE_GROUP = 8

    def _init_slices(self, slice_poses):
        """Per-slice rigid transforms (Sec. 3.3.2): every slice of every stack is a one-slice
        grid (inputs.slice_grids) with its own pose, a rotation R about the slice's centre and a
        translation tau; slice_poses optionally gives the starting (R, tau) of each, stacks in
        order, slices in order.  The slices are binned in groups of
        SLICE_GROUP grids, each group rendering into its slices' rows of the stack tensors."""
        c = self.cfg
        if c.nrf is not None or c.lambda_ssim > 0 or c.progressive or c.block_radius:
            raise ValueError("per-slice poses run the plain smooth-L1 method only")
        self.slices = []          # (stack, slice) of every slice grid, in order
        nominal = []
        for k, st in enumerate(self.stacks):
            for z, g in enumerate(inputs.slice_grids(st)):
                self.slices.append((k, z))
                nominal.append(g)
        # each slice rotates about its own centre, where rotation and translation decouple
        self.poses = [rigid.StackPose(g, centre=rigid.grid_centre(g)) for g in nominal]
        if slice_poses is not None:
            if len(slice_poses) != len(self.poses):
                raise ValueError("one (R, tau) per slice")
            for q, (R, tau) in zip(self.poses, slice_poses):
                q.R = np.asarray(R, np.float64).copy()
                q.tau = np.asarray(tau, np.float64).copy()
        frozen = [i for i, (k, _) in enumerate(self.slices) if k in set(c.pose_frozen)]
        self.pose_opt = rigid.PoseAdam(self.poses, c.lr_pose_rot, c.lr_pose_trans, frozen=frozen)
        n = self.p.n
        self.groups = []
        for i0 in range(0, len(nominal), self.SLICE_GROUP):
            idx = list(range(i0, min(i0 + self.SLICE_GROUP, len(nominal))))
            self.groups.append((self._bins(n, [nominal[i] for i in idx], 10), idx))
        self.bins = None
        self.slice_out = [self.outs[k][z:z + 1] for k, z in self.slices]
        self.slice_dl = [self.dls[k][z:z + 1] for k, z in self.slices]
        self.grads = api.GaussParams.zeros_like(self.p)

    def _step_slices(self):
        """One iteration with per-slice poses: each group of slice grids is binned and
        rendered, the smooth-L1 term is formed over the whole stacks, then each group's
        backward partials give its slices' affine gradients and accumulate the chain rule (the
        anisotropy term once), and Adam steps the Gaussians and the slice poses."""
        c = self.cfg
        grids = [q.grid() for q in self.poses]
        for b, idx in self.groups:
            b.set_grids([grids[i] for i in idx])
            b.bin(self.p)
            api.render(b, list(range(len(idx))), [self.slice_out[i] for i in idx])
        loss, _ = api.smooth_l1(self.outs, self.targets, self.dls)
        for t in self.grads.tensors():
            t.zero_()
        G = []
        for gi, (b, idx) in enumerate(self.groups):
            ids = list(range(len(idx)))
            api.grid_partials(self.p, b, ids, [self.slice_dl[i] for i in idx])
            G.append(api.pose_grads(self.p, b, ids))
            api.chain(self.p, b, ids, self.grads, c.lambda_aniso if gi == 0 else 0.0, c.lambda_r)
        self.pose_opt.step(list(torch.cat(G).cpu().numpy().reshape(-1, 3, 4)))
        for prm, gr, mm, vv, lr in zip(self.p.tensors(), self.grads.tensors(), self.m.tensors(),
                                       self.v.tensors(), self.lrs()):
            api.adam_step(prm, gr, mm, vv, lr, self.it - self.adam_t0)
        return loss

    def _bins(self, n, grids, per):
        c = self.cfg
        return api.Bins(n, grids, capacity=int(per * n * len(grids)) + 4096,
                        block_radius=c.block_radius, cell_resolution=c.cell_resolution)

    def lrs(self):
        c = self.cfg
        return (c.lr_mean, c.lr_quat, c.lr_scale, c.lr_logit)

    def refine(self, g_new: int):
        """Replace the lattice by the g_new^3 lattice interpolated from it."""
        self.p = api.upsample_lattice(self.p, self.lattice, g_new)
        self.lattice = g_new
        self.m = api.GaussParams.zeros_like(self.p)
        self.v = api.GaussParams.zeros_like(self.p)
        self.bins = self._bins(self.p.n, self.bins.grids, 10)
        if self.vbins is not None:
            self.vbins = self._bins(self.p.n, [self.volume_grid], 12)
        self.adam_t0 = self.it

    def step(self) -> torch.Tensor:
        c = self.cfg
        for done, g_new in c.progressive:
            if done == self.it:
                self.refine(g_new)
        self.it += 1
        if self.slices is not None:
            return self._step_slices()
        if c.nrf is not None and not self.nrf_on and self.it > int(c.nrf_start * c.n_iter):
            self.nrf_on = True
        if self.poses is not None:
            self.bins.set_grids([q.grid() for q in self.poses])
        self.bins.bin(self.p)
        # the loss is formed in the render's epilogue (with the residual field added to every
        # voxel first once it is on); the renderings are stored only when the SSIM term reads
        # them
        loss, _ = api.render_loss(self.bins, self.ids, self.targets, self.dls,
                                  outs=self.outs if c.lambda_ssim > 0 else None,
                                  nrf=c.nrf if self.nrf_on else None)
        if c.lambda_ssim > 0:
            loss = loss + c.lambda_ssim * api.ssim_loss(self.outs, self.targets, self.dls,
                                                        c.lambda_ssim)
        api.grid_partials(self.p, self.bins, self.ids, self.dls)
        if self.poses is not None:
            G = api.pose_grads(self.p, self.bins, self.ids).cpu().numpy()
            self.pose_opt.step(list(G))
        if self.nrf_on:
            c.nrf.zero_grad()
            c.nrf.backward_grids(self.stacks, self.dls, n_sample=c.nrf_sample)
            c.nrf.adam_step(c.lr_nrf)
        # chain rule and Adam on the four groups in one pass: the parameters change only here,
        # after everything above has read them
        api.chain_adam(self.p, self.bins, self.ids, self.m, self.v, self.lrs(),
                       self.it - self.adam_t0, c.lambda_aniso, c.lambda_r)
        return loss

    def render_volume(self) -> torch.Tensor:
        self.vbins.bin(self.p)
        return api.render_volume(self.vbins, 0, nrf=self.cfg.nrf if self.nrf_on else None)

    def psnr(self) -> float:
        vol = self.render_volume()
        mse = float(api.mse(vol, self.phantom))
        return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)

    def run(self, n_iter: Optional[int] = None, log=None) -> List[dict]:
        n_iter = self.cfg.n_iter if n_iter is None else n_iter
        hist = []
        if self.phantom is not None:
            hist.append({"it": self.it, "loss": None, "psnr": self.psnr()})
        for _ in range(n_iter):
            loss = self.step()
            if self.phantom is not None and (self.it % self.cfg.psnr_every == 0):
                rec = {"it": self.it, "loss": float(loss), "psnr": self.psnr()}
                hist.append(rec)
                if log:
                    log(rec)
        return hist


def iters_to_psnr(hist: List[dict], target: float) -> Optional[int]:
    """First logged iteration whose PSNR reaches target (None if never)."""
    for rec in hist:
        if rec["psnr"] is not None and rec["psnr"] >= target:
            return rec["it"]
    return None

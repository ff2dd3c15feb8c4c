"""Tensor-level wrappers over the C ABI.  PyTorch supplies device memory and the stream; every
step of the computation runs in libgm's HIP kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import GmError, check, load, ptr_array


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t: torch.Tensor, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclasses.dataclass
class GaussParams:
    """Device tensors of the Gaussian parameters (Eq. 2-3): mean [N,3], quat [N,4],
    log_scale [N,3], logit [N], float32."""
    mean: torch.Tensor
    quat: torch.Tensor
    log_scale: torch.Tensor
    logit: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    @staticmethod
    def from_host(g, device="cuda") -> "GaussParams":
        return GaussParams(*(torch.from_numpy(np.ascontiguousarray(getattr(g, k), np.float32))
                             .to(device) for k in ("mean", "quat", "log_scale", "logit")))

    # set by zeros_like: the one buffer the four tensors are views of
    flat: Optional[torch.Tensor] = dataclasses.field(default=None, repr=False, compare=False)

    @staticmethod
    def zeros_like(p: "GaussParams") -> "GaussParams":
        """Zeroed tensors of p's shapes, laid out back to back in one buffer so that
        zero_() clears them with a single fill."""
        # each tensor starts on a 256-byte boundary (the kernels read quaternions as float4)
        sizes = [t.numel() for t in p.tensors()]
        starts = []
        o = 0
        for k in sizes:
            starts.append(o)
            o += -(-k // 64) * 64
        flat = torch.zeros(max(o, 1), dtype=torch.float32, device=p.mean.device)
        views = [flat[a:a + k].view(t.shape) for a, k, t in zip(starts, sizes, p.tensors())]
        return GaussParams(*views, flat=flat)

    def zero_(self):
        if self.flat is not None:
            self.flat.zero_()
        else:
            for t in self.tensors():
                t.zero_()
        return self

    def tensors(self):
        return (self.mean, self.quat, self.log_scale, self.logit)

    def struct(self) -> _lib.GmGaussians:
        for t, nm in zip(self.tensors(), ("mean", "quat", "log_scale", "logit")):
            _need(t, torch.float32, nm)
        return _lib.GmGaussians(self.n, _p(self.mean), _p(self.quat), _p(self.log_scale),
                                _p(self.logit))

    def grad_struct(self) -> _lib.GmGrads:
        for t, nm in zip(self.tensors(), ("mean", "quat", "log_scale", "logit")):
            _need(t, torch.float32, nm)
        return _lib.GmGrads(self.n, _p(self.mean), _p(self.quat), _p(self.log_scale),
                            _p(self.logit))


_WS = {}


def workspace(device=None) -> torch.Tensor:
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    if dev not in _WS:
        _WS[dev] = torch.empty(_lib.GM_REDUCE_WORKSPACE_BYTES // 4, dtype=torch.float32,
                               device=dev)
    return _WS[dev]


class Bins:
    """Binning state for n Gaussians on a fixed list of grids (gm_bins).  Device buffers are
    torch tensors owned by this object; the pair capacity grows on demand."""

    def __init__(self, n: int, grids: Sequence, capacity: Optional[int] = None,
                 cutoff: float = 3.0, device="cuda", block_radius: int = 0,
                 cell_resolution: int = 0):
        load()
        self.grids = list(grids)
        self.n = int(n)
        self.cutoff = float(cutoff)
        # block_radius > 0: the paper's cell-neighbourhood query (Eqs. 4-6) instead of the box
        self.block_radius = int(block_radius)
        self.cell_resolution = int(cell_resolution)
        self.device = torch.device(device)
        self._cgrids = (_lib.GmGrid * len(self.grids))(*[_lib.grid_struct(g) for g in self.grids])
        rb = ctypes.c_size_t()
        tt = ctypes.c_int64()
        check(load().gm_bin_query(self.n, self._cgrids, len(self.grids), 0, ctypes.byref(rb),
                                  ctypes.byref(tt), None))
        self.total_tiles = int(tt.value)
        G = len(self.grids)
        dev = self.device
        self.records = torch.empty((G, max(self.n, 1), 16), dtype=torch.float32, device=dev)
        self.tile_count = torch.empty((G, max(self.n, 1)), dtype=torch.int32, device=dev)
        self.box_volume = torch.zeros(max(G, 2), dtype=torch.int64, device=dev)
        self.tile_start = torch.empty(self.total_tiles + 1, dtype=torch.int32, device=dev)
        self.grid_grads = torch.empty((G, max(self.n, 1), 10), dtype=torch.float32, device=dev)
        # one FP64 loss partial per tile for the fused render + loss
        self.loss_part = torch.empty(max(self.total_tiles, 1), dtype=torch.float64, device=dev)
        self.capacity = 0
        self.pair_gauss = None
        self.scratch = None
        self._reserve(capacity if capacity is not None else max(1024, 8 * self.n * G))
        self.n_pairs = -1
        # bumped by every bin(): records, lists and partials describe the parameters of the
        # last bin() only, so a saved generation tells whether they still hold
        self.generation = 0

    def _reserve(self, cap: int):
        cap = int(min(cap, 2 ** 31 - 1))
        sb = ctypes.c_size_t()
        check(load().gm_bin_query(self.n, self._cgrids, len(self.grids), cap, None, None,
                                  ctypes.byref(sb)))
        self.pair_gauss = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        self.scratch = torch.empty((int(sb.value) + 3) // 4, dtype=torch.int32, device=self.device)
        self.capacity = cap

    def struct(self) -> _lib.GmBins:
        if hasattr(self, "_s"):
            b = self._s
        else:
            b = _lib.GmBins()
            b.n_pairs = -1       # not yet filled by gm_bin
        b.n_grids = len(self.grids)
        b.n_gauss = self.n
        b.capacity_pairs = self.capacity
        b.records = _p(self.records)
        b.tile_count = _p(self.tile_count)
        b.box_volume = _p(self.box_volume)
        b.tile_start = _p(self.tile_start)
        b.pair_gauss = _p(self.pair_gauss)
        b.grid_grads = _p(self.grid_grads)
        b.scratch = _p(self.scratch)
        b.scratch_bytes = self.scratch.numel() * 4
        self._s = b
        return b

    def bin(self, g: GaussParams, allow_nonfinite: bool = False) -> int:
        if g.n != self.n:
            raise ValueError(f"bins built for {self.n} Gaussians, got {g.n}")
        gs = g.struct()
        self.generation += 1
        opts = _lib.GmBinOpts(self.cutoff, self.block_radius, self.cell_resolution)
        npairs = ctypes.c_int64()
        for _ in range(2):
            b = self.struct()
            st = load().gm_bin(ctypes.byref(gs), self._cgrids, len(self.grids), ctypes.byref(opts),
                               ctypes.byref(b), ctypes.byref(npairs), _stream())
            if st == _lib.GM_ERR_CAPACITY:
                self._reserve(int(npairs.value * 1.25) + 1024)
                continue
            if st == _lib.GM_ERR_NONFINITE and allow_nonfinite:
                break
            check(st)
            break
        self.n_pairs = int(npairs.value)
        return self.n_pairs

    def set_grids(self, grids: Sequence):
        """Replace the grids' affines (and slice profiles) for the next bin(); the dimensions
        must stay those the buffers were sized for."""
        grids = list(grids)
        if len(grids) != len(self.grids) or any(
                (a.nx, a.ny, a.nz) != (b.nx, b.ny, b.nz) for a, b in zip(grids, self.grids)):
            raise ValueError("set_grids keeps the number and dimensions of the grids")
        self.grids = grids
        self._cgrids = (_lib.GmGrid * len(grids))(*[_lib.grid_struct(g) for g in grids])
        self.generation += 1
        self.n_pairs = -1
        if hasattr(self, "_s"):
            self._s.n_pairs = -1

    @property
    def tile_base_host(self):
        """Global id of each grid's first tile (filled by gm_bin)."""
        return [int(self._s.tile_base[k]) for k in range(len(self.grids) + 1)]

    # -- views for tests -------------------------------------------------------------------
    def boxes(self, k: int):
        r = self.records[k, :self.n].view(torch.int32)
        return r[:, 10:13], r[:, 13:16]

    def pair_count(self, k: Optional[int] = None) -> int:
        """Contributing (Gaussian, voxel) pairs of the last bin() (read from the device)."""
        v = self.box_volume[:len(self.grids)].cpu()
        return int(v.sum()) if k is None else int(v[k])

    @property
    def box_pairs_host(self) -> List[int]:
        """Contributing pairs per grid of the last bin(), as gm_bin reported them (no device
        access)."""
        return [int(self._s.box_pairs[k]) for k in range(len(self.grids))]


def render(bins: Bins, ids: Sequence[int], outs: Optional[List[torch.Tensor]] = None):
    """gm_render_stacks on the listed grids; returns the rendered [nz,ny,nx] tensors."""
    if outs is None:
        outs = [torch.empty(bins.grids[i].shape, dtype=torch.float32, device=bins.device)
                for i in ids]
    for t in outs:
        _need(t, torch.float32, "out")
    idarr = (ctypes.c_int32 * max(1, len(ids)))(*ids)
    check(load().gm_render_stacks(ctypes.byref(bins.struct()), idarr, len(ids),
                                  ptr_array([t.data_ptr() for t in outs]), _stream()))
    return outs


def render_loss(bins: Bins, ids: Sequence[int], targets: Sequence[torch.Tensor],
                dl_di: Optional[List[torch.Tensor]] = None,
                outs: Optional[List[torch.Tensor]] = None, nrf=None):
    """gm_render_loss_smooth_l1: renders the listed grids and forms the smooth-L1 term in the
    same pass; returns (loss device scalar, dL/dI per stack).  The renderings are stored only
    when outs is given.  With nrf (an nrf.NRF), gm_render_nrf_loss_smooth_l1: the residual
    field is added to every voxel in the same pass before the loss."""
    if dl_di is None:
        dl_di = [torch.empty_like(t) for t in targets]
    for t in list(targets) + list(dl_di) + list(outs or []):
        _need(t, torch.float32, "render-loss operand")
    for i, t, d in zip(ids, targets, dl_di):
        shp = tuple(bins.grids[i].shape)
        if tuple(t.shape) != shp or tuple(d.shape) != shp:
            raise ValueError(f"grid {i}: target / dl_di shape differs from {shp}")
    if outs is not None and len(outs) != len(ids):
        raise ValueError("outs must hold one tensor per listed grid")
    loss = torch.empty(4, dtype=torch.float32, device=bins.device)
    idarr = (ctypes.c_int32 * max(1, len(ids)))(*ids)
    out_arr = None if outs is None else ptr_array([t.data_ptr() for t in outs])
    if nrf is None:
        check(load().gm_render_loss_smooth_l1(
            ctypes.byref(bins.struct()), idarr, len(ids),
            ptr_array([t.data_ptr() for t in targets]), out_arr,
            ptr_array([d.data_ptr() for d in dl_di]), _p(loss), _p(bins.loss_part),
            bins.loss_part.numel() * 8, _stream()))
    else:
        check(load().gm_render_nrf_loss_smooth_l1(
            ctypes.byref(bins.struct()), idarr, len(ids), ctypes.byref(nrf.struct()),
            ptr_array([t.data_ptr() for t in targets]), out_arr,
            ptr_array([d.data_ptr() for d in dl_di]), _p(loss), _p(bins.loss_part),
            bins.loss_part.numel() * 8, _stream()))
    return loss[0], dl_di


def render_volume(bins: Bins, grid_id: int, out: Optional[torch.Tensor] = None, nrf=None):
    if out is None:
        out = torch.empty(bins.grids[grid_id].shape, dtype=torch.float32, device=bins.device)
    _need(out, torch.float32, "out")
    nrf_s = None if nrf is None else ctypes.byref(nrf.struct())
    check(load().gm_render_volume(ctypes.byref(bins.struct()), int(grid_id), nrf_s, _p(out),
                                  _stream()))
    return out


def backward(g: GaussParams, bins: Bins, ids: Sequence[int], dl_di: Sequence[torch.Tensor],
             grads: GaussParams, lambda_aniso: float = 0.0, lambda_r: float = 1.5):
    """gm_backward: accumulates (+=) into grads."""
    for t in dl_di:
        _need(t, torch.float32, "dl_di")
    idarr = (ctypes.c_int32 * max(1, len(ids)))(*ids)
    gs = g.struct()
    gr = grads.grad_struct()
    check(load().gm_backward(ctypes.byref(gs), ctypes.byref(bins.struct()), idarr, len(ids),
                             ptr_array([t.data_ptr() for t in dl_di]), float(lambda_aniso),
                             float(lambda_r), ctypes.byref(gr), _stream()))
    return grads


def grid_partials(g: GaussParams, bins: Bins, ids: Sequence[int], dl_di: Sequence[torch.Tensor]):
    """gm_grid_partials: the first stage of backward(); fills bins.grid_grads for ids."""
    for t in dl_di:
        _need(t, torch.float32, "dl_di")
    idarr = (ctypes.c_int32 * max(1, len(ids)))(*ids)
    gs = g.struct()
    check(load().gm_grid_partials(ctypes.byref(gs), ctypes.byref(bins.struct()), idarr, len(ids),
                                  ptr_array([t.data_ptr() for t in dl_di]), _stream()))
    return bins.grid_grads


def chain(g: GaussParams, bins: Bins, ids: Sequence[int], grads: GaussParams,
          lambda_aniso: float = 0.0, lambda_r: float = 1.5):
    """gm_chain: the second stage of backward(); accumulates (+=) into grads."""
    idarr = (ctypes.c_int32 * max(1, len(ids)))(*ids)
    gs = g.struct()
    gr = grads.grad_struct()
    check(load().gm_chain(ctypes.byref(gs), ctypes.byref(bins.struct()), idarr, len(ids),
                          float(lambda_aniso), float(lambda_r), ctypes.byref(gr), _stream()))
    return grads


def chain_adam(g: GaussParams, bins: Bins, ids: Sequence[int], m: GaussParams, v: GaussParams,
               lrs: Sequence[float], step: int, lambda_aniso: float = 0.0,
               lambda_r: float = 1.5, beta1: float = 0.9, beta2: float = 0.999,
               eps: float = 1e-8):
    """gm_chain_adam: chain rule and Adam in one pass; g, m and v are updated in place.
    lrs: learning rates of the mean, quat, log_scale and logit groups."""
    if len(lrs) != 4:
        raise ValueError("four learning rates: mean, quat, log_scale, logit")
    idarr = (ctypes.c_int32 * max(1, len(ids)))(*ids)
    gs = g.struct()
    ms, vs = m.grad_struct(), v.grad_struct()
    opts = _lib.GmAdamOpts((ctypes.c_double * 4)(*[float(x) for x in lrs]), float(beta1),
                           float(beta2), float(eps), int(step))
    check(load().gm_chain_adam(ctypes.byref(gs), ctypes.byref(bins.struct()), idarr, len(ids),
                               float(lambda_aniso), float(lambda_r), ctypes.byref(opts),
                               ctypes.byref(ms), ctypes.byref(vs), _stream()))
    return g


def smooth_l1(preds: Sequence[torch.Tensor], targets: Sequence[torch.Tensor],
              dl_di: Optional[List[torch.Tensor]] = None):
    """gm_loss_smooth_l1: returns (loss device scalar, dL/dI per stack)."""
    if dl_di is None:
        dl_di = [torch.empty_like(p) for p in preds]
    for t in list(preds) + list(targets) + list(dl_di):
        _need(t, torch.float32, "loss operand")
    loss = torch.empty(4, dtype=torch.float32, device=preds[0].device)
    sizes = (ctypes.c_int64 * len(preds))(*[p.numel() for p in preds])
    check(load().gm_loss_smooth_l1(len(preds), ptr_array([p.data_ptr() for p in preds]),
                                   ptr_array([t.data_ptr() for t in targets]), sizes,
                                   ptr_array([d.data_ptr() for d in dl_di]), _p(loss),
                                   _p(workspace()), _stream()))
    return loss[0], dl_di


def upsample_lattice(g: GaussParams, g_old: int, g_new: int) -> GaussParams:
    """gm_upsample_lattice: the g_new^3 lattice interpolated from the g_old^3 one."""
    n = g_new ** 3
    dev = g.mean.device
    out = GaussParams(torch.empty((n, 3), device=dev), torch.empty((n, 4), device=dev),
                      torch.empty((n, 3), device=dev), torch.empty(n, device=dev))
    gs = g.struct()
    check(load().gm_upsample_lattice(int(g_old), ctypes.byref(gs), int(g_new), _p(out.mean),
                                     _p(out.quat), _p(out.log_scale), _p(out.logit), _stream()))
    return out


def pose_grads(g: GaussParams, bins: Bins, ids: Sequence[int]) -> torch.Tensor:
    """gm_grid_pose_grads: dL/d(world->index affine) [len(ids), 3, 4] (float64, device) of the
    objective whose partials the last backward / grid_partials call on these bins left."""
    out = torch.empty((max(1, len(ids)), 12), dtype=torch.float64, device=bins.device)
    nbytes = 256 * max(1, len(ids)) * 12 * 8
    ws = torch.empty(nbytes // 8, dtype=torch.float64, device=bins.device)
    idarr = (ctypes.c_int32 * max(1, len(ids)))(*ids)
    gs = g.struct()
    check(load().gm_grid_pose_grads(ctypes.byref(gs), ctypes.byref(bins.struct()), idarr,
                                    len(ids), _p(out), _p(ws), nbytes, _stream()))
    return out[:len(ids)].view(-1, 3, 4)


def ssim_loss(preds: Sequence[torch.Tensor], targets: Sequence[torch.Tensor],
              dl_di: Sequence[torch.Tensor], lam: float = 0.5):
    """gm_loss_ssim: L_SSIM = 1 - mean SSIM over every slice of every [nz, ny, nx] stack
    (device scalar); dl_di[k] += lam * dL_SSIM/dpred_k."""
    for t in list(preds) + list(targets) + list(dl_di):
        _need(t, torch.float32, "loss operand")
    for p, t, d in zip(preds, targets, dl_di):
        if p.dim() != 3 or t.shape != p.shape or d.shape != p.shape:
            raise ValueError("SSIM operands must be [nz, ny, nx] stacks of equal shape")
    loss = torch.empty(4, dtype=torch.float32, device=preds[0].device)
    dims = (ctypes.c_int32 * (3 * len(preds)))(
        *[v for p in preds for v in (p.shape[2], p.shape[1], p.shape[0])])
    check(load().gm_loss_ssim(len(preds), ptr_array([p.data_ptr() for p in preds]),
                              ptr_array([t.data_ptr() for t in targets]), dims, float(lam),
                              ptr_array([d.data_ptr() for d in dl_di]), _p(loss),
                              _p(workspace()), _stream()))
    return loss[0]


def aniso(g: GaussParams, lambda_r: float = 1.5):
    val = torch.empty(4, dtype=torch.float32, device=g.mean.device)
    gs = g.struct()
    check(load().gm_aniso_reg(ctypes.byref(gs), float(lambda_r), _p(val), _p(workspace()),
                              _stream()))
    return val[0]


def adam_step(p: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr: float,
              step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    for t, nm in ((p, "param"), (g, "grad"), (m, "m"), (v, "v")):
        _need(t, torch.float32, nm)
    check(load().gm_adam_step(_p(p), _p(g), _p(m), _p(v), p.numel(), float(lr), float(beta1),
                              float(beta2), float(eps), int(step), _stream()))


def mse(vol: torch.Tensor, ref: torch.Tensor):
    _need(vol, torch.float32, "vol")
    _need(ref, torch.float32, "ref")
    out = torch.empty(4, dtype=torch.float32, device=vol.device)
    check(load().gm_mse(_p(vol), _p(ref), vol.numel(), _p(out), _p(workspace()), _stream()))
    return out[0]


def devox_init(g: int, stacks, stack_data: Sequence[torch.Tensor]) -> GaussParams:
    """gm_devox_init: g^3 Gaussians on a uniform grid initialised from the stacks."""
    n = g ** 3
    dev = stack_data[0].device
    for t in stack_data:
        _need(t, torch.float32, "stack data")
    p = GaussParams(torch.empty((n, 3), device=dev), torch.empty((n, 4), device=dev),
                    torch.empty((n, 3), device=dev), torch.empty((n,), device=dev))
    cg = (_lib.GmGrid * len(stacks))(*[_lib.grid_struct(s) for s in stacks])
    check(load().gm_devox_init(int(g), cg, len(stacks), ptr_array([t.data_ptr() for t in stack_data]),
                               _p(p.mean), _p(p.quat), _p(p.log_scale), _p(p.logit), _stream()))
    return p

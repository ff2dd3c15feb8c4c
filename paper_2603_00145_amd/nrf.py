"""Neural residual field (Sec. 3.4, Eq. 8) on the HIP path: FP32 master weights and Adam
moments, BF16 copies for the MFMA kernels, forward / backward through the C ABI."""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import numpy as np
import torch

from . import _lib, api
from ._lib import check, load


class NRF:
    """r(x) = out_scale tanh(w_out . a_D + b_out), a_l = SiLU(W_l a_{l-1} + b_l),
    a_0 = (x, sin(2^k pi x), cos(2^k pi x), k < n_freq).  width 64."""

    def __init__(self, n_freq: int = 16, depth: int = 3, out_scale: float = 0.1, seed: int = 0,
                 zero_last: bool = True, device="cuda"):
        self.n_freq, self.depth, self.width, self.out_scale = n_freq, depth, 64, out_scale
        self.in_dim = 3 + 6 * n_freq
        # the kernels encode bands in groups of four: 64 inputs hold 8 bands, 128 hold 20
        self.in_pad = 64 if n_freq <= 8 else 128
        if not 0 <= n_freq <= 20:
            raise ValueError("n_freq must lie in [0, 20]")
        dev = torch.device(device)
        rng = np.random.default_rng(seed)
        Wd = self.width

        def unif(shape, fan_in):
            b = 1.0 / math.sqrt(fan_in)
            return rng.uniform(-b, b, size=shape).astype(np.float32)

        w_in = np.zeros((Wd, self.in_pad), np.float32)
        w_in[:, :self.in_dim] = unif((Wd, self.in_dim), self.in_dim)
        params = {
            "w_in": w_in, "b_in": unif((Wd,), self.in_dim),
            "w_hid": unif((max(depth - 1, 1), Wd, Wd), Wd), "b_hid": unif((max(depth - 1, 1), Wd), Wd),
            "w_out": np.zeros(Wd, np.float32) if zero_last else unif((Wd,), Wd),
            "b_out": np.zeros(1, np.float32) if zero_last else unif((1,), Wd),
        }
        self.p = {k: torch.from_numpy(v).to(dev).contiguous() for k, v in params.items()}
        self.g = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.bf = {k: torch.empty(self.p[k].shape, dtype=torch.int16, device=dev)
                   for k in ("w_in", "w_hid", "w_out")}
        self.step_no = 0
        self._ws = None
        self.sync_bf16()

    # -- C structs ------------------------------------------------------------------------
    def struct(self) -> _lib.GmNrf:
        s = _lib.GmNrf()
        s.n_freq, s.depth, s.width, s.in_pad = self.n_freq, self.depth, self.width, self.in_pad
        s.out_scale = self.out_scale
        s.w_in, s.b_in = self.bf["w_in"].data_ptr(), self.p["b_in"].data_ptr()
        s.w_hid, s.b_hid = self.bf["w_hid"].data_ptr(), self.p["b_hid"].data_ptr()
        s.w_out, s.b_out = self.bf["w_out"].data_ptr(), self.p["b_out"].data_ptr()
        self._s = s
        return s

    def grads_struct(self) -> _lib.GmNrfGrads:
        g = self.g
        return _lib.GmNrfGrads(g["w_in"].data_ptr(), g["b_in"].data_ptr(), g["w_hid"].data_ptr(),
                               g["b_hid"].data_ptr(), g["w_out"].data_ptr(), g["b_out"].data_ptr())

    # -- operations -----------------------------------------------------------------------
    def sync_bf16(self):
        for k, t in self.bf.items():
            check(load().gm_f32_to_bf16(ctypes.c_void_p(self.p[k].data_ptr()),
                                        ctypes.c_void_p(t.data_ptr()), t.numel(), api._stream()))

    def forward_add(self, grid, out: torch.Tensor):
        """out[v] += r(x_v) for every voxel of grid."""
        api._need(out, torch.float32, "out")
        check(load().gm_nrf_forward(ctypes.byref(self.struct()), ctypes.byref(_lib.grid_struct(grid)),
                                    ctypes.c_void_p(out.data_ptr()), api._stream()))

    def zero_grad(self):
        for t in self.g.values():
            t.zero_()

    def backward(self, grid, dl_dr: torch.Tensor, idx: Optional[torch.Tensor] = None,
                 n_sample: Optional[int] = None, generator: Optional[torch.Generator] = None):
        """Accumulate the gradient of scale * sum_k dl_dr[v_k] r(x_{v_k}) over the voxels
        v_k = idx (default: n_sample uniform random voxels, scale = voxels / n_sample)."""
        api._need(dl_dr, torch.float32, "dl_dr")
        nvox = grid.n_voxels
        if idx is None and n_sample is not None and n_sample < nvox:
            idx = torch.randint(0, nvox, (n_sample,), device=dl_dr.device, dtype=torch.int32,
                                generator=generator)
        npts = nvox if idx is None else int(idx.numel())
        scale = nvox / npts if idx is not None and npts > 0 else 1.0
        nb = ctypes.c_size_t()
        s = self.struct()
        check(load().gm_nrf_workspace(ctypes.byref(s), npts, ctypes.byref(nb)))
        if self._ws is None or self._ws.numel() * 4 < nb.value:
            self._ws = torch.empty((nb.value + 3) // 4, dtype=torch.float32, device=dl_dr.device)
        gs = self.grads_struct()
        check(load().gm_nrf_backward(ctypes.byref(s), ctypes.byref(_lib.grid_struct(grid)),
                                     ctypes.c_void_p(0 if idx is None else idx.data_ptr()), npts,
                                     ctypes.c_void_p(dl_dr.data_ptr()), float(scale),
                                     ctypes.byref(gs), ctypes.c_void_p(self._ws.data_ptr()),
                                     self._ws.numel() * 4, api._stream()))
        return idx, scale

    def backward_grids(self, grids, dls, idxs=None, n_sample: Optional[int] = None,
                       generator: Optional[torch.Generator] = None):
        """backward over several grids in one call (one chain pass per grid, the weight
        gradients over all the points at once): the gradient of sum over grids k of
        scale_k * sum_j dls[k][v_kj] r(x_{v_kj}), point lists as for backward."""
        n = len(grids)
        if n != len(dls) or (idxs is not None and len(idxs) != n):
            raise ValueError("grids, dls and idxs differ in length")
        idx_l, npts, scales = [], [], []
        for k, (grid, dl) in enumerate(zip(grids, dls)):
            api._need(dl, torch.float32, "dl_dr")
            nvox = grid.n_voxels
            idx = None if idxs is None else idxs[k]
            if idx is None and n_sample is not None and n_sample < nvox:
                idx = torch.randint(0, nvox, (n_sample,), device=dl.device, dtype=torch.int32,
                                    generator=generator)
            idx_l.append(idx)
            npts.append(nvox if idx is None else int(idx.numel()))
            scales.append(nvox / npts[-1] if idx is not None and npts[-1] > 0 else 1.0)
        s = self.struct()
        n_pts = (ctypes.c_int64 * n)(*npts)
        nb = ctypes.c_size_t()
        check(load().gm_nrf_workspace_grids(ctypes.byref(s), n, n_pts, ctypes.byref(nb)))
        if self._ws is None or self._ws.numel() * 4 < nb.value:
            self._ws = torch.empty((nb.value + 3) // 4, dtype=torch.float32, device=dls[0].device)
        gs = self.grads_struct()
        structs = (_lib.GmGrid * n)(*[_lib.grid_struct(g) for g in grids])
        ptr = ctypes.c_void_p
        idx_p = (ptr * n)(*[ptr(0 if i is None else i.data_ptr()) for i in idx_l])
        dl_p = (ptr * n)(*[ptr(d.data_ptr()) for d in dls])
        sc = (ctypes.c_float * n)(*scales)
        check(load().gm_nrf_backward_grids(ctypes.byref(s), n, structs, idx_p, n_pts, dl_p, sc,
                                           ctypes.byref(gs), ptr(self._ws.data_ptr()),
                                           self._ws.numel() * 4, api._stream()))
        return idx_l, scales

    def adam_step(self, lr: float = 1e-4):
        self.step_no += 1
        for k in self.p:
            api.adam_step(self.p[k], self.g[k], self.m[k], self.v[k], lr, self.step_no)
        self.sync_bf16()

    def weights_host(self):
        """BF16-valued weights as float64 numpy arrays (for the oracle)."""
        def bf(t):
            u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
            return u.view(np.float32).astype(np.float64)
        W = [bf(self.bf["w_in"])] + [bf(self.bf["w_hid"])[l] for l in range(self.depth - 1)]
        b = [self.p["b_in"].cpu().numpy().astype(np.float64)] + \
            [self.p["b_hid"].cpu().numpy().astype(np.float64)[l] for l in range(self.depth - 1)]
        return {"W": W, "b": b, "w_out": bf(self.bf["w_out"]),
                "b_out": float(self.p["b_out"].cpu().numpy()[0])}

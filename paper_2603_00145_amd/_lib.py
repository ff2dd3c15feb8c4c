"""ctypes binding of libgm.so (include/gm.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgm.so")

GM_MAX_GRIDS = 8
ABI_VERSION = 5          # struct layouts of include/gm.h this binding mirrors
GM_RECORD_FLOATS = 16
GM_GRID_GRAD_FLOATS = 10
GM_REDUCE_WORKSPACE_BYTES = 16384
GM_NOALLOC_MAX_TILES = 131072

STATUS = {0: "GM_OK", 1: "GM_ERR_INVALID_ARGUMENT", 2: "GM_ERR_CAPACITY",
          3: "GM_ERR_NONFINITE", 4: "GM_ERR_HIP", 5: "GM_ERR_UNSUPPORTED"}
GM_OK, GM_ERR_INVALID_ARGUMENT, GM_ERR_CAPACITY, GM_ERR_NONFINITE, GM_ERR_HIP, \
    GM_ERR_UNSUPPORTED = range(6)


class GmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


P = ctypes.c_void_p


class GmGaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean", P), ("quat", P), ("log_scale", P), ("logit", P)]


class GmGrads(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean", P), ("quat", P), ("log_scale", P), ("logit", P)]


class GmGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("world_to_index", ctypes.c_double * 12),
                ("psf_sigma_z", ctypes.c_double)]


class GmBinOpts(ctypes.Structure):
    _fields_ = [("cutoff_sigma", ctypes.c_double), ("block_radius", ctypes.c_int32),
                ("cell_resolution", ctypes.c_int32)]


class GmAdamOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double * 4), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double), ("step", ctypes.c_int32)]


class GmBins(ctypes.Structure):
    _fields_ = [("n_grids", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_gauss", ctypes.c_int64), ("capacity_pairs", ctypes.c_int64),
                ("records", P), ("tile_count", P), ("box_volume", P), ("tile_start", P),
                ("pair_gauss", P), ("grid_grads", P), ("scratch", P),
                ("scratch_bytes", ctypes.c_size_t),
                ("grids", GmGrid * GM_MAX_GRIDS),
                ("tile_base", ctypes.c_int64 * (GM_MAX_GRIDS + 1)),
                ("n_pairs", ctypes.c_int64), ("box_pairs", ctypes.c_int64 * GM_MAX_GRIDS),
                ("list_start", ctypes.c_int64 * (GM_MAX_GRIDS + 1)),
                ("cutoff_sigma", ctypes.c_double), ("block_radius", ctypes.c_int32),
                ("cell_resolution", ctypes.c_int32)]


class GmNrfGrads(ctypes.Structure):
    _fields_ = [("w_in", P), ("b_in", P), ("w_hid", P), ("b_hid", P), ("w_out", P), ("b_out", P)]


class GmWsNet(ctypes.Structure):
    _fields_ = [("w", P * 4), ("b", P * 4), ("wl", P), ("bl", P)]


class GmWsGrads(ctypes.Structure):
    _fields_ = [("w", P * 4), ("b", P * 4), ("wl", P), ("bl", P)]


class GmNrf(ctypes.Structure):
    _fields_ = [("n_freq", ctypes.c_int32), ("depth", ctypes.c_int32), ("width", ctypes.c_int32),
                ("in_pad", ctypes.c_int32), ("out_scale", ctypes.c_float),
                ("reserved", ctypes.c_int32), ("w_in", P), ("b_in", P), ("w_hid", P),
                ("b_hid", P), ("w_out", P), ("b_out", P)]


# (name, restype, argtypes); entry points declared in include/gm.h
_SIGS = [
    ("gm_abi_version", ctypes.c_int32, []),
    ("gm_last_error", ctypes.c_char_p, []),
    ("gm_tile_dims", None, [ctypes.POINTER(ctypes.c_int32)]),
    ("gm_bin_query", ctypes.c_int, [ctypes.c_int64, ctypes.POINTER(GmGrid), ctypes.c_int32,
                                     ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_size_t)]),
    ("gm_bin", ctypes.c_int, [ctypes.POINTER(GmGaussians), ctypes.POINTER(GmGrid),
                               ctypes.c_int32, ctypes.POINTER(GmBinOpts),
                               ctypes.POINTER(GmBins), ctypes.POINTER(ctypes.c_int64), P]),
    ("gm_render_stacks", ctypes.c_int, [ctypes.POINTER(GmBins), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.c_int32, ctypes.POINTER(P), P]),
    ("gm_render_loss_smooth_l1", ctypes.c_int,
     [ctypes.POINTER(GmBins), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.POINTER(P),
      ctypes.POINTER(P), ctypes.POINTER(P), P, P, ctypes.c_size_t, P]),
    ("gm_render_loss_smooth_l1_noalloc", ctypes.c_int,
     [ctypes.POINTER(GmBins), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.POINTER(P),
      ctypes.POINTER(P), ctypes.POINTER(P), P, P]),
    ("gm_render_volume", ctypes.c_int, [ctypes.POINTER(GmBins), ctypes.c_int32,
                                         ctypes.POINTER(GmNrf), P, P]),
    ("gm_render_nrf_loss_smooth_l1", ctypes.c_int,
     [ctypes.POINTER(GmBins), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
      ctypes.POINTER(GmNrf), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), P, P,
      ctypes.c_size_t, P]),
    ("gm_loss_smooth_l1", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(P),
                                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(P), P,
                                          P, P]),
    ("gm_grid_pose_grads", ctypes.c_int, [ctypes.POINTER(GmGaussians), ctypes.POINTER(GmBins),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, P, P,
                                           ctypes.c_size_t, P]),
    ("gm_upsample_lattice", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(GmGaussians),
                                            ctypes.c_int32, P, P, P, P, P]),
    ("gm_loss_ssim", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(P),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.c_float,
                                     ctypes.POINTER(P), P, P, P]),
    ("gm_aniso_reg", ctypes.c_int, [ctypes.POINTER(GmGaussians), ctypes.c_float, P, P, P]),
    ("gm_backward", ctypes.c_int, [ctypes.POINTER(GmGaussians), ctypes.POINTER(GmBins),
                                    ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                    ctypes.POINTER(P), ctypes.c_float, ctypes.c_float,
                                    ctypes.POINTER(GmGrads), P]),
    ("gm_grid_partials", ctypes.c_int, [ctypes.POINTER(GmGaussians), ctypes.POINTER(GmBins),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                         ctypes.POINTER(P), P]),
    ("gm_chain", ctypes.c_int, [ctypes.POINTER(GmGaussians), ctypes.POINTER(GmBins),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_float,
                                 ctypes.c_float, ctypes.POINTER(GmGrads), P]),
    ("gm_chain_adam", ctypes.c_int, [ctypes.POINTER(GmGaussians), ctypes.POINTER(GmBins),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                      ctypes.c_float, ctypes.c_float, ctypes.POINTER(GmAdamOpts),
                                      ctypes.POINTER(GmGrads), ctypes.POINTER(GmGrads), P]),
    ("gm_adam_step", ctypes.c_int, [P, P, P, P, ctypes.c_int64, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int32, P]),
    ("gm_mse", ctypes.c_int, [P, P, ctypes.c_int64, P, P, P]),
    ("gm_index_to_world", ctypes.c_int, [ctypes.POINTER(GmGrid), ctypes.POINTER(ctypes.c_double)]),
    ("gm_nrf_forward", ctypes.c_int, [ctypes.POINTER(GmNrf), ctypes.POINTER(GmGrid), P, P]),
    ("gm_nrf_workspace", ctypes.c_int, [ctypes.POINTER(GmNrf), ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_size_t)]),
    ("gm_nrf_backward", ctypes.c_int, [ctypes.POINTER(GmNrf), ctypes.POINTER(GmGrid), P,
                                        ctypes.c_int64, P, ctypes.c_float,
                                        ctypes.POINTER(GmNrfGrads), P, ctypes.c_size_t, P]),
    ("gm_nrf_workspace_grids", ctypes.c_int, [ctypes.POINTER(GmNrf), ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_size_t)]),
    ("gm_nrf_backward_grids", ctypes.c_int, [ctypes.POINTER(GmNrf), ctypes.c_int32,
                                              ctypes.POINTER(GmGrid), ctypes.POINTER(P),
                                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(P),
                                              ctypes.POINTER(ctypes.c_float),
                                              ctypes.POINTER(GmNrfGrads), P, ctypes.c_size_t, P]),
    ("gm_f32_to_bf16", ctypes.c_int, [P, P, ctypes.c_int64, P]),
    ("gm_ws_gather", ctypes.c_int, [ctypes.POINTER(GmGrid), ctypes.c_int32, ctypes.POINTER(P), P,
                                     ctypes.c_int64, ctypes.c_float, P, P]),
    ("gm_ws_targets", ctypes.c_int, [P, P, ctypes.c_int64, P, P]),
    ("gm_ws_workspace", ctypes.c_int, [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    ("gm_ws_forward", ctypes.c_int, [ctypes.POINTER(GmWsNet), P, ctypes.c_int64, P, P, P, P, P,
                                      P, ctypes.c_size_t, P]),
    ("gm_ws_backward", ctypes.c_int, [ctypes.POINTER(GmWsNet), P, ctypes.c_int64, P, P, P, P, P,
                                       ctypes.POINTER(GmWsGrads), P, ctypes.c_size_t, P]),
    ("gm_devox_init", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(GmGrid), ctypes.c_int32,
                                      ctypes.POINTER(P), P, P, P, P, P]),
]

EXPORTED = [s[0] for s in _SIGS]

_lib = None


def load(path: str = LIB_PATH):
    """Load libgm.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as "
                           "g; g.build()'` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.gm_abi_version() != ABI_VERSION:
        raise RuntimeError(f"libgm ABI version {lib.gm_abi_version()}, binding expects {ABI_VERSION}")
    _lib = lib
    return lib


def check(status: int):
    if status != GM_OK:
        raise GmError(status, load().gm_last_error().decode())


def ptr_array(ptrs):
    arr = (P * max(1, len(ptrs)))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr


def grid_struct(g) -> GmGrid:
    s = GmGrid()
    s.nx, s.ny, s.nz = int(g.nx), int(g.ny), int(g.nz)
    A = [float(v) for v in g.world_to_index.reshape(-1)]
    for i in range(12):
        s.world_to_index[i] = A[i]
    s.psf_sigma_z = float(g.psf_sigma_z)
    return s


def tile_dims():
    out = (ctypes.c_int32 * 3)()
    load().gm_tile_dims(out)
    return tuple(out)


def index_to_world(g):
    """The library's index->world affine (3x4 float64) of a grid descriptor."""
    import numpy as np
    out = (ctypes.c_double * 12)()
    check(load().gm_index_to_world(ctypes.byref(grid_struct(g)), out))
    return np.array(list(out)).reshape(3, 4)

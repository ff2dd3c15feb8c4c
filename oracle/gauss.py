"""Plain FP64 definitions of Magnetic-Gaussian rendering on voxel grids and its gradients.

Test infrastructure only (see the package docstring).

The model (paper Sec. 3.2-3.3): a Gaussian G_i = {mu_i, Sigma_i, alpha_i} (Eq. 2) with
Sigma = R S S^T R^T, S = diag(exp s), R from the normalised quaternion (Eq. 3), contributes
alpha_i exp(-1/2 (x - mu_i)^T Sigma_i^-1 (x - mu_i)) to the intensity at x (Eq. 7).

Evaluated on a grid g with world->index affine [L | t] at integer voxel index v, in the
grid's index frame:
    c = L mu + t,   Sigma_idx = L Sigma L^T.
Stacks carry a Gaussian slice profile of std-dev sig along index z (the slice normal); the
recorded value is the Gaussian convolved with that normalised 1D profile, which is again a
Gaussian with
    Sigma_g = Sigma_idx + sig^2 e_z e_z^T,   amp = alpha sqrt(det Sigma_idx / det Sigma_g),
so  I_g[v] = sum_i 1[v in Box_g(i)] amp_i exp(-1/2 (v - c_i)^T Sigma_g,i^-1 (v - c_i)).
With sig = 0 this is Eq. 7 at voxel centres.  Box_g(i) comes from oracle.recipe.
alpha = sigmoid(logit) keeps the intensity in [0, 1] (Eq. 2 states alpha in [0, 1]).

Everything here is computed in float64 from the float32 inputs; functions taking
``dtype`` also run in complex128 for complex-step differentiation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

from . import recipe

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(os.path.dirname(__file__), "_build", "libbrute.so")
        if not os.path.exists(path):
            from . import build
            build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        lib.oracle_render.argtypes = [I, I, I, I, P, P, P, P, P, P, P]
        lib.oracle_render_points.argtypes = [I, P, I, P, P, P, P, P, P, P]
        lib.oracle_partials.argtypes = [I, I, I, I, P, P, P, P, P, P, P, P, P, P]
        lib.oracle_render.restype = None
        lib.oracle_render_points.restype = None
        lib.oracle_partials.restype = None
        lib.oracle_scatter_render.argtypes = [I, I, I, I, P, P, P, P, P, P, P]
        lib.oracle_scatter_render.restype = None
        lib.oracle_render_cells.argtypes = [I, I, I, I, P, P, P, P, P, P, I, P]
        lib.oracle_render_cells.restype = None
        lib.oracle_partials_cells.argtypes = [I, I, I, I, P, P, P, P, P, P, I, P, P, P, P]
        lib.oracle_render_points_cells.argtypes = [I, P, P, I, P, P, P, P, P, I, P]
        lib.oracle_render_points_cells.restype = None
        lib.oracle_partials_cells.restype = None
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _LIB = lib
    return _LIB


def threads() -> int:
    """OpenMP threads the brute-force sums run on."""
    return int(_lib().oracle_threads())


def set_threads(k: int) -> None:
    """Thread count of the brute-force sums (k <= 0: unchanged)."""
    _lib().oracle_set_threads(int(k))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------------------
# per-Gaussian quantities (Eq. 2-3, slice profile)
# ----------------------------------------------------------------------------------------

def quat_to_rot(qn):
    """Hamilton rotation matrix of unit quaternions qn[..., (w,x,y,z)]; columns are the
    rotated coordinate axes."""
    w, x, y, z = qn[..., 0], qn[..., 1], qn[..., 2], qn[..., 3]
    R = np.empty(qn.shape[:-1] + (3, 3), dtype=qn.dtype)
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def sigmoid(a):
    return 1.0 / (1.0 + np.exp(-a))


def params64(g, dtype=np.float64):
    """(mean, quat, log_scale, logit) of a Gaussians object as arrays of ``dtype``."""
    return tuple(np.asarray(getattr(g, k), np.float32).astype(np.float64).astype(dtype)
                 for k in ("mean", "quat", "log_scale", "logit"))


def world_terms(mean, quat, log_scale, logit):
    """World-space quantities: normalised quaternion, R, S^2 = exp(2 s), Sigma, alpha."""
    qnorm = np.sqrt((quat * quat).sum(-1))
    qn = quat / qnorm[:, None]
    R = quat_to_rot(qn)
    S2 = np.exp(2 * log_scale)
    Sigma = np.einsum("nij,nj,nkj->nik", R, S2, R)
    alpha = sigmoid(logit)
    return dict(qnorm=qnorm, qn=qn, R=R, S2=S2, Sigma=Sigma, alpha=alpha)


def grid_terms(mean, quat, log_scale, logit, grid, wt=None):
    """Index-frame quantities on one grid: centre c, Sigma_idx, Sigma_g, conic C =
    Sigma_g^-1 and amplitude amp (slice-profile convolution in closed form)."""
    if wt is None:
        wt = world_terms(mean, quat, log_scale, logit)
    A = np.asarray(grid.world_to_index)
    A = A if np.iscomplexobj(A) else A.astype(np.float64)   # complex for complex-step checks
    L, t = A[:, :3], A[:, 3]
    c = mean @ L.T + t
    Sig_idx = np.einsum("ij,njk,lk->nil", L, wt["Sigma"], L)
    Sig_g = Sig_idx.copy()
    Sig_g[:, 2, 2] = Sig_g[:, 2, 2] + grid.psf_sigma_z ** 2
    C = np.linalg.inv(Sig_g)
    amp = wt["alpha"] * np.sqrt(np.linalg.det(Sig_idx) / np.linalg.det(Sig_g))
    return dict(c=c, Sig_idx=Sig_idx, Sig_g=Sig_g, C=C, amp=amp, L=L, wt=wt)


# ----------------------------------------------------------------------------------------
# rendering
# ----------------------------------------------------------------------------------------

def _f64c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _boxes_c(lo, hi, nonempty):
    return (np.ascontiguousarray(lo, np.int64), np.ascontiguousarray(hi, np.int64),
            np.ascontiguousarray(nonempty, np.uint8))


def render(grid, gt, lo, hi, nonempty):
    """Brute force FP64 over every voxel and every Gaussian (ascending i), box-tested."""
    lib = _lib()
    n = gt["c"].shape[0]
    out = np.zeros(grid.shape, np.float64)
    c, C, amp = _f64c(gt["c"]), _f64c(gt["C"]), _f64c(gt["amp"])
    lo, hi, ne = _boxes_c(lo, hi, nonempty)
    lib.oracle_render(grid.nx, grid.ny, grid.nz, n, _ptr(c), _ptr(C), _ptr(amp), _ptr(lo),
                      _ptr(hi), _ptr(ne), _ptr(out))
    return out


def render_scatter(grid, gt, lo, hi, nonempty):
    """The same sums as render(), each Gaussian visiting its own box (ascending i per voxel, so
    the result is identical); its cost is the box volumes, so it serves full-size grids."""
    lib = _lib()
    n = gt["c"].shape[0]
    out = np.zeros(grid.shape, np.float64)
    c, C, amp = _f64c(gt["c"]), _f64c(gt["C"]), _f64c(gt["amp"])
    lo, hi, ne = _boxes_c(lo, hi, nonempty)
    lib.oracle_scatter_render(grid.nx, grid.ny, grid.nz, n, _ptr(c), _ptr(C), _ptr(amp),
                              _ptr(lo), _ptr(hi), _ptr(ne), _ptr(out))
    return out


def render_points(points, gt, lo, hi, nonempty):
    """Values at selected voxels points[k] = (x, y, z), brute force over all Gaussians."""
    lib = _lib()
    pts = np.ascontiguousarray(points, np.int64)
    n = gt["c"].shape[0]
    out = np.zeros(pts.shape[0], np.float64)
    c, C, amp = _f64c(gt["c"]), _f64c(gt["C"]), _f64c(gt["amp"])
    lo, hi, ne = _boxes_c(lo, hi, nonempty)
    lib.oracle_render_points(pts.shape[0], _ptr(pts), n, _ptr(c), _ptr(C), _ptr(amp),
                             _ptr(lo), _ptr(hi), _ptr(ne), _ptr(out))
    return out


def render_numpy(grid, gt, lo, hi, nonempty):
    """Same sum as render(), vectorised in numpy for tiny inputs; works in complex128."""
    dt = np.result_type(gt["c"].dtype, gt["C"].dtype, gt["amp"].dtype)
    z, y, x = np.meshgrid(np.arange(grid.nz), np.arange(grid.ny), np.arange(grid.nx),
                          indexing="ij")
    v = np.stack([x, y, z], -1).reshape(-1, 3).astype(np.float64)
    out = np.zeros(v.shape[0], dtype=dt)
    for i in range(gt["c"].shape[0]):
        if not nonempty[i]:
            continue
        inside = ((v >= lo[i]) & (v <= hi[i])).all(1)
        d = v[inside] - gt["c"][i]
        q = np.einsum("kj,jl,kl->k", d, gt["C"][i], d)
        out[inside] = out[inside] + gt["amp"][i] * np.exp(-0.5 * q)
    return out.reshape(grid.shape)


def render_cells(grid, gt, vcell, gcell, valid, radius):
    """render() with the paper's block query (Sec. 3.3.1, Eqs. 4-6) in place of the box:
    voxel v takes Gaussian i when valid[i] and |vcell[v] - gcell[i]| <= radius on every world
    axis (vcell from recipe.voxel_cells, gcell from recipe.mean_cells).  Brute force over
    every voxel and every Gaussian, ascending i."""
    lib = _lib()
    n = gt["c"].shape[0]
    out = np.zeros(grid.shape, np.float64)
    c, C, amp = _f64c(gt["c"]), _f64c(gt["C"]), _f64c(gt["amp"])
    vc = np.ascontiguousarray(vcell, np.int64).reshape(-1, 3)
    gc = np.ascontiguousarray(gcell, np.int64).reshape(-1, 3)
    va = np.ascontiguousarray(valid, np.uint8)
    assert vc.shape[0] == grid.n_voxels and gc.shape[0] == n and va.shape[0] == n
    lib.oracle_render_cells(grid.nx, grid.ny, grid.nz, n, _ptr(c), _ptr(C), _ptr(amp), _ptr(vc),
                            _ptr(gc), _ptr(va), int(radius), _ptr(out))
    return out


def render_points_cells(points, pcell, gt, gcell, valid, radius):
    """render_cells at selected voxels points[k] = (x, y, z) whose world positions have the
    cells pcell[k] (recipe.voxel_cells of those voxels), brute force over all Gaussians."""
    lib = _lib()
    pts = np.ascontiguousarray(points, np.int64).reshape(-1, 3)
    pc = np.ascontiguousarray(pcell, np.int64).reshape(-1, 3)
    n = gt["c"].shape[0]
    out = np.zeros(pts.shape[0], np.float64)
    c, C, amp = _f64c(gt["c"]), _f64c(gt["C"]), _f64c(gt["amp"])
    gc = np.ascontiguousarray(gcell, np.int64).reshape(-1, 3)
    va = np.ascontiguousarray(valid, np.uint8)
    assert pc.shape[0] == pts.shape[0] and gc.shape[0] == n and va.shape[0] == n
    lib.oracle_render_points_cells(pts.shape[0], _ptr(pts), _ptr(pc), n, _ptr(c), _ptr(C),
                                   _ptr(amp), _ptr(gc), _ptr(va), int(radius), _ptr(out))
    return out


# ----------------------------------------------------------------------------------------
# gradients
# ----------------------------------------------------------------------------------------

def grid_partials(grid, gt, lo, hi, nonempty, dl_di):
    """Per-Gaussian sums over its box of the derivatives of sum_v dl_di[v] I[v] with respect
    to the grid-frame quantities: d_amp [N], d_c [N,3] and G_C [N,3,3] = dL/dC (C taken as
    a full matrix; symmetric)."""
    lib = _lib()
    n = gt["c"].shape[0]
    c, C, amp = _f64c(gt["c"]), _f64c(gt["C"]), _f64c(gt["amp"])
    lo, hi, ne = _boxes_c(lo, hi, nonempty)
    g = _f64c(dl_di)
    d_amp = np.zeros(n)
    d_c = np.zeros((n, 3))
    G_C = np.zeros((n, 3, 3))
    lib.oracle_partials(grid.nx, grid.ny, grid.nz, n, _ptr(c), _ptr(C), _ptr(amp), _ptr(lo),
                        _ptr(hi), _ptr(ne), _ptr(g), _ptr(d_amp), _ptr(d_c), _ptr(G_C))
    return d_amp, d_c, G_C


def grid_partials_cells(grid, gt, vcell, gcell, valid, radius, dl_di):
    """grid_partials() over the voxels the block query gives each Gaussian (render_cells)."""
    lib = _lib()
    n = gt["c"].shape[0]
    c, C, amp = _f64c(gt["c"]), _f64c(gt["C"]), _f64c(gt["amp"])
    vc = np.ascontiguousarray(vcell, np.int64).reshape(-1, 3)
    gc = np.ascontiguousarray(gcell, np.int64).reshape(-1, 3)
    va = np.ascontiguousarray(valid, np.uint8)
    assert vc.shape[0] == grid.n_voxels and gc.shape[0] == n and va.shape[0] == n
    g = _f64c(dl_di)
    d_amp = np.zeros(n)
    d_c = np.zeros((n, 3))
    G_C = np.zeros((n, 3, 3))
    lib.oracle_partials_cells(grid.nx, grid.ny, grid.nz, n, _ptr(c), _ptr(C), _ptr(amp),
                              _ptr(vc), _ptr(gc), _ptr(va), int(radius), _ptr(g), _ptr(d_amp),
                              _ptr(d_c), _ptr(G_C))
    return d_amp, d_c, G_C


def sigma_idx_grad(gt, d_amp, G_C):
    """dL/dSigma_idx per Gaussian from the grid-frame partials: the conic C = Sigma_g^-1 gives
    dL/dSigma_g = -C G_C C, and amp = alpha sqrt(det Sigma_idx / det Sigma_g) adds
    -1/2 d_amp amp C (through Sigma_g) and +1/2 d_amp amp Sigma_idx^-1; Sigma_g = Sigma_idx
    + sig^2 e_z e_z^T, so dSigma_g = dSigma_idx."""
    C = gt["C"]
    ha = 0.5 * (d_amp * gt["amp"])[:, None, None]
    G_g = -np.einsum("nij,njk,nkl->nil", C, G_C, C) - ha * C
    return G_g + ha * np.linalg.inv(gt["Sig_idx"])


def pose_grad(mean, quat, log_scale, logit, grid, partial):
    """Gradient of the objective behind one grid's partials (d_amp, d_c, G_C) with respect to
    the grid's world->index affine A = [L | t] (row-major 3x4), boxes held fixed: the
    quantity a joint optimisation of the stacks' rigid transforms T_k (Sec. 3.3.2) chains
    through.  c = L mu + t gives dL/dL = sum_i d_c,i mu_i^T and dL/dt = sum_i d_c,i;
    Sigma_idx = L Sigma L^T gives dL/dL += sum_i 2 G_idx,i L Sigma_i (G_idx symmetric)."""
    d_amp, d_c, G_C = partial
    wt = world_terms(mean, quat, log_scale, logit)
    gt = grid_terms(mean, quat, log_scale, logit, grid, wt)
    G_idx = sigma_idx_grad(gt, d_amp, G_C)
    G_L = np.einsum("ni,nj->ij", d_c, mean) + \
        2 * np.einsum("nij,jk,nkl->il", G_idx, gt["L"], wt["Sigma"])
    G_t = d_c.sum(0)
    return np.concatenate([G_L, G_t[:, None]], axis=1)


def chain(mean, quat, log_scale, logit, grids, partials):
    """Raw-parameter gradients from the grid-frame partials of every grid.

    Per grid: dL/dmu += L^T d_c;  dL/dSigma_g = -C G_C C;  log amp = log alpha
    + 1/2 log det Sigma_idx - 1/2 log det Sigma_g gives dL/dSigma_idx = dL/dSigma_g
    + 1/2 d_amp amp Sigma_idx^-1 - ... (the Sigma_g part: -1/2 d_amp amp C), and
    dL/dSigma += L^T dL/dSigma_idx L;  dL/dalpha += d_amp amp / alpha.
    Then Sigma = R diag(e^2s) R^T: dL/dR = 2 G R D, dL/ds_m = 2 e^{2 s_m} (R^T G R)_mm;
    R(q_hat) by the Hamilton formula; q_hat = q/|q|; alpha = sigmoid(logit).
    """
    wt = world_terms(mean, quat, log_scale, logit)
    n = mean.shape[0]
    dt = np.result_type(mean.dtype, np.float64)
    d_mu = np.zeros((n, 3), dt)
    G_S = np.zeros((n, 3, 3), dt)
    d_alpha = np.zeros(n, dt)
    for grid, (d_amp, d_c, G_C) in zip(grids, partials):
        gt = grid_terms(mean, quat, log_scale, logit, grid, wt)
        L = gt["L"]
        d_mu += d_c @ L
        G_idx = sigma_idx_grad(gt, d_amp, G_C)
        G_S += np.einsum("ji,njk,kl->nil", L, G_idx, L)
        d_alpha += d_amp * gt["amp"] / wt["alpha"]
    R, S2 = wt["R"], wt["S2"]
    GR = 2 * np.einsum("nij,njk,nk->nik", G_S, R, S2)
    RtGR = np.einsum("nji,njk,nkl->nil", R, G_S, R)
    d_s = 2 * S2 * np.einsum("nii->ni", RtGR)
    qn = wt["qn"]
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    g = GR
    d_qn = np.stack([
        2 * (-z * g[:, 0, 1] + y * g[:, 0, 2] + z * g[:, 1, 0] - x * g[:, 1, 2]
             - y * g[:, 2, 0] + x * g[:, 2, 1]),
        2 * (y * g[:, 0, 1] + z * g[:, 0, 2] + y * g[:, 1, 0] - 2 * x * g[:, 1, 1]
             - w * g[:, 1, 2] + z * g[:, 2, 0] + w * g[:, 2, 1] - 2 * x * g[:, 2, 2]),
        2 * (-2 * y * g[:, 0, 0] + x * g[:, 0, 1] + w * g[:, 0, 2] + x * g[:, 1, 0]
             + z * g[:, 1, 2] - w * g[:, 2, 0] + z * g[:, 2, 1] - 2 * y * g[:, 2, 2]),
        2 * (-2 * z * g[:, 0, 0] - w * g[:, 0, 1] + x * g[:, 0, 2] + w * g[:, 1, 0]
             - 2 * z * g[:, 1, 1] + y * g[:, 1, 2] + x * g[:, 2, 0] + y * g[:, 2, 1]),
    ], axis=1)
    d_q = (d_qn - qn * (qn * d_qn).sum(1, keepdims=True)) / wt["qnorm"][:, None]
    d_logit = d_alpha * wt["alpha"] * (1 - wt["alpha"])
    return d_mu, d_q, d_s, d_logit


def aniso(log_scale, lam_r):
    """Eq. 13 with the ratio of the actual scales: mean_i max(0, e^{max s - min s} - lam_r).
    Gradient: +-e^D/N on the first argmax / first argmin where the hinge is active."""
    s = np.asarray(log_scale, np.float32).astype(np.float64)
    n = s.shape[0]
    if n == 0:
        return 0.0, np.zeros_like(s)
    imax = np.argmax(s, axis=1)
    imin = np.argmin(s, axis=1)
    D = s[np.arange(n), imax] - s[np.arange(n), imin]
    ratio = np.exp(D)
    act = ratio > lam_r
    val = float(np.where(act, ratio - lam_r, 0.0).sum() / n)
    grad = np.zeros_like(s)
    gr = np.where(act, ratio / n, 0.0)
    np.add.at(grad, (np.arange(n), imax), gr)
    np.add.at(grad, (np.arange(n), imin), -gr)
    return val, grad


def smooth_l1(preds: Sequence[np.ndarray], targets: Sequence[np.ndarray]):
    """Eq. 11 (beta = 1) averaged over every voxel of every stack; returns the value and
    dL/dI per stack."""
    ntot = sum(p.size for p in preds)
    val = 0.0
    grads = []
    for p, y in zip(preds, targets):
        d = np.asarray(p, np.float64) - np.asarray(y, np.float64)
        ad = np.abs(d)
        val += float(np.where(ad < 1.0, 0.5 * d * d, ad - 0.5).sum())
        grads.append(np.clip(d, -1.0, 1.0) / ntot)
    return val / ntot, grads


def adam(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in the PyTorch arrangement, FP64.  Returns (param, m, v)."""
    p = np.asarray(param, np.float64)
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    bc1 = 1 - beta1 ** step
    bc2 = 1 - beta2 ** step
    p = p - (lr / bc1) * m / (np.sqrt(v) / np.sqrt(bc2) + eps)
    return p, m, v


def psnr(vol, ref):
    mse = float(np.mean((np.asarray(vol, np.float64) - np.asarray(ref, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


# ----------------------------------------------------------------------------------------
# convenience: everything for one set of Gaussians on several grids
# ----------------------------------------------------------------------------------------

def prepare(g, grids, cutoff=3.0):
    """Per grid: (terms, lo, hi, nonempty, valid) for a Gaussians object."""
    mean, quat, ls, logit = params64(g)
    wt = world_terms(mean, quat, ls, logit)
    out = []
    for gr in grids:
        lo, hi, ne, valid = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, gr, cutoff)
        gt = grid_terms(mean, quat, ls, logit, gr, wt)
        out.append((gt, lo, hi, ne, valid))
    return out


def render_all(g, grids, cutoff=3.0):
    return [render(gr, gt, lo, hi, ne) for gr, (gt, lo, hi, ne, _) in
            zip(grids, prepare(g, grids, cutoff))]


def gradients(g, grids, dl_dis, cutoff=3.0, lam_aniso=0.0, lam_r=1.5):
    """Analytic FP64 raw-parameter gradients of sum_g sum_v dl_di_g[v] I_g[v]
    (+ lam_aniso * aniso loss), boxes held fixed."""
    mean, quat, ls, logit = params64(g)
    prep = prepare(g, grids, cutoff)
    parts = [grid_partials(gr, gt, lo, hi, ne, d) for gr, (gt, lo, hi, ne, _), d in
             zip(grids, prep, dl_dis)]
    d_mu, d_q, d_s, d_a = chain(mean, quat, ls, logit, grids, parts)
    if lam_aniso:
        d_s = d_s + lam_aniso * aniso(g.log_scale, lam_r)[1]
    return d_mu, d_q, d_s, d_a


# ----------------------------------------------------------------------------------------
# devoxelization initialisation (Sec. 3.1, Fig. 1b)
# ----------------------------------------------------------------------------------------

def _trilinear_index(vol, p):
    """Trilinear value of vol[z,y,x] at index point p = (x, y, z) inside [0, n-1]^3."""
    nz, ny, nx = vol.shape
    x0 = min(int(np.floor(p[0])), max(nx - 2, 0))
    y0 = min(int(np.floor(p[1])), max(ny - 2, 0))
    z0 = min(int(np.floor(p[2])), max(nz - 2, 0))
    x1, y1, z1 = min(x0 + 1, nx - 1), min(y0 + 1, ny - 1), min(z0 + 1, nz - 1)
    fx, fy, fz = p[0] - x0, p[1] - y0, p[2] - z0
    v = np.asarray(vol, np.float64)
    c = 0.0
    for zz, wz in ((z0, 1 - fz), (z1, fz)):
        for yy, wy in ((y0, 1 - fy), (y1, fy)):
            for xx, wx in ((x0, 1 - fx), (x1, fx)):
                c += wz * wy * wx * v[zz, yy, xx]
    return c


def devox_init(g, stacks, stack_data):
    """g^3 Gaussians at the cell centres of [-1,1]^3, identity rotation, sigma = h/2, and
    alpha = clip(mean over the stacks whose index domain contains the centre of the stack
    sampled trilinearly there, times h^3 / ((2 pi)^{3/2} sigma^3), 1e-3, 1 - 1e-3).
    Returns (mean, quat, log_scale, logit) in float64."""
    h = 2.0 / g
    sigma = h / 2
    pu = h ** 3 / ((2 * np.pi) ** 1.5 * sigma ** 3)
    n = g ** 3
    mean = np.zeros((n, 3))
    logit = np.zeros(n)
    for i in range(n):
        ix, iy, iz = i % g, (i // g) % g, i // (g * g)
        x = np.array([-1 + (2 * ix + 1) / g, -1 + (2 * iy + 1) / g, -1 + (2 * iz + 1) / g])
        mean[i] = x
        vals = []
        for grid, data in zip(stacks, stack_data):
            A = np.asarray(grid.world_to_index, np.float64)
            p = A[:, :3] @ x + A[:, 3]
            if np.all(p >= 0) and p[0] <= grid.nx - 1 and p[1] <= grid.ny - 1 and p[2] <= grid.nz - 1:
                vals.append(_trilinear_index(data, p))
        v = np.mean(vals) if vals else 0.0
        a = min(max(v * pu, 1e-3), 1 - 1e-3)
        logit[i] = np.log(a / (1 - a))
    quat = np.zeros((n, 4))
    quat[:, 0] = 1
    log_scale = np.full((n, 3), np.log(sigma))
    return mean, quat, log_scale, logit


# ----------------------------------------------------------------------------------------
# sensitivity of the gradients to the per-voxel upstream gradient
# ----------------------------------------------------------------------------------------

def abs_jacobian_sums(g, grids, cutoff=3.0, chunk=1 << 20):
    """For every raw parameter component theta of every Gaussian i: sum over the grids and over
    the voxels v of Box_g(i) of |d w_i(v) / d theta|, where w_i(v) is the Gaussian's value at v
    (the term of I_g[v], Eq. 7 with the slice profile).  The gradient of sum_v dl[v] I[v]
    changes by at most max_v |delta dl[v]| times this sum when dl changes by delta dl.

    Per pair: d w / d amp = w / amp, d w / d c = w C delta, d w / d C_aa = -1/2 w delta_a^2,
    d w / d C_ab = -w delta_a delta_b (a < b, both symmetric entries), delta = v - c; the
    derivatives of (amp, c, C) with respect to the raw parameters come from complex-step
    differentiation of grid_terms.  Returns (mean [N,3], quat [N,4], log_scale [N,3],
    logit [N])."""
    n = g.mean.shape[0]
    p64 = params64(g)
    sizes = (3, 4, 3, 1)
    out = [np.zeros((n, k)) for k in sizes]
    h = 1e-30
    for grid in grids:
        lo, hi, ne, _ = recipe.boxes(g.mean, g.quat, g.log_scale, g.logit, grid, cutoff)
        gt = grid_terms(*p64, grid)
        # Jacobian of (amp, c0..2, C00 C11 C22 C01 C02 C12) with respect to the 11 raw components
        J = np.zeros((n, 10, 11))
        col = 0
        for grp, k in enumerate(sizes):
            for comp in range(k):
                pc = [np.asarray(a, np.complex128).copy() for a in p64]
                if pc[grp].ndim == 1:
                    pc[grp] = pc[grp] + 1j * h
                else:
                    pc[grp][:, comp] = pc[grp][:, comp] + 1j * h
                t = grid_terms(*pc, grid)
                C = t["C"]
                J[:, 0, col] = t["amp"].imag / h
                J[:, 1:4, col] = t["c"].imag / h
                J[:, 4:10, col] = np.stack([C[:, 0, 0], C[:, 1, 1], C[:, 2, 2], C[:, 0, 1],
                                            C[:, 0, 2], C[:, 1, 2]], 1).imag / h
                col += 1
        idx = np.nonzero(ne)[0]
        dims = (hi[idx] - lo[idx] + 1).astype(np.int64)
        cnt = np.prod(dims, axis=1)
        acc = np.zeros((n, 11))
        # enumerate the box voxels of the nonempty Gaussians in chunks of whole Gaussians
        starts = np.concatenate([[0], np.cumsum(cnt)])
        a = 0
        while a < idx.size:
            b = int(np.searchsorted(starts, starts[a] + chunk, side="right")) - 1
            b = max(b, a + 1)
            sel = idx[a:b]
            c_sel = cnt[a:b]
            gi = np.repeat(sel, c_sel)
            k = np.arange(int(c_sel.sum())) - np.repeat(starts[a:b] - starts[a], c_sel)
            d = dims[a:b]
            dx, dy = np.repeat(d[:, 0], c_sel), np.repeat(d[:, 1], c_sel)
            vx = lo[gi, 0] + k % dx
            vy = lo[gi, 1] + (k // dx) % dy
            vz = lo[gi, 2] + k // (dx * dy)
            delta = np.stack([vx, vy, vz], 1).astype(np.float64) - gt["c"][gi]
            Cg = gt["C"][gi]
            Cd = np.einsum("pij,pj->pi", Cg, delta)
            q = (delta * Cd).sum(1)
            e = np.exp(-0.5 * q)
            w = gt["amp"][gi] * e
            dw = np.empty((gi.size, 10))
            dw[:, 0] = e
            dw[:, 1:4] = w[:, None] * Cd
            dw[:, 4] = -0.5 * w * delta[:, 0] ** 2
            dw[:, 5] = -0.5 * w * delta[:, 1] ** 2
            dw[:, 6] = -0.5 * w * delta[:, 2] ** 2
            dw[:, 7] = -w * delta[:, 0] * delta[:, 1]
            dw[:, 8] = -w * delta[:, 0] * delta[:, 2]
            dw[:, 9] = -w * delta[:, 1] * delta[:, 2]
            jt = np.abs(np.einsum("pk,pkl->pl", dw, J[gi]))
            for col in range(11):
                acc[:, col] += np.bincount(gi, weights=jt[:, col], minlength=n)
            a = b
        col = 0
        for grp, k in enumerate(sizes):
            out[grp] += acc[:, col:col + k]
            col += k
    out[3] = out[3][:, 0]
    return tuple(out)

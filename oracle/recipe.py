"""The box recipe: which voxels of a grid a Gaussian is evaluated on (FP64, numpy).

Which voxels belong to a Gaussian's truncation box is an integer decision taken from
floating point, so it is made by one fixed recipe in IEEE binary64 (round to nearest even,
no fused multiply-add, correctly rounded sqrt and division, operations in the order
written below).  numpy float64 ufuncs are exactly that.  The HIP path implements the same
recipe independently; the two agree bit for bit.

The box replaces the paper's cell-neighbourhood query (Sec. 3.3.1, Eqs. 4-6) by an
axis-aligned box of +-cutoff standard deviations of the Gaussian's marginals in each grid's
index frame, including the slice profile on stacks.  Every voxel with Mahalanobis distance
<= cutoff lies inside it.

Recipe, per (Gaussian, grid) with world->index affine [L | t] and slice sigma sig:
  1. n2 = ((w*w + x*x) + y*y) + z*z; invalid unless n2 > 0, n2 finite and every input
     finite; q_hat = q / sqrt(n2) component-wise.  (Also invalid: an e_m of step 3 that
     is 0 or infinite.)
  2. R from q_hat (Hamilton, (w,x,y,z)), each entry as  1 - 2*(a*a + b*b)  or
     2*(a*b -+ c*d)  in exactly that association.
  3. e_m = exp_recipe(s_m) (below).
  4. M_jm = ((L_j0*R_0m + L_j1*R_1m) + L_j2*R_2m);  B_jm = M_jm * e_m.
  5. D_j = ((B_j0*B_j0 + B_j1*B_j1) + B_j2*B_j2);  D_2 = D_2 + sig*sig;
     rho_j = cutoff * sqrt(D_j).
  6. c_j = ((L_j0*mu_0 + L_j1*mu_1) + L_j2*mu_2) + t_j.
  7. lo_j = ceil(c_j - rho_j), hi_j = floor(c_j + rho_j), each clamped to [-2^30, 2^30]
     (a NaN lo becomes +2^30 and a NaN hi -2^30, i.e. an empty box);
     then lo_j = max(lo_j, 0), hi_j = min(hi_j, n_j - 1); empty if lo_j > hi_j on any
     axis or the input was invalid.
  8. Tiles touched: [lo_j // T_j, hi_j // T_j] for tile edge T_j.

block_boxes() is the paper's own rule instead (Eqs. 4-6, cells of [-1, 1]^3 within a block
radius of the Gaussian's cell), for grids whose world->index map is axis-aligned.  On any
grid, rotated stacks included, voxel_cells() and mean_cells() give the cells the rule
compares: a voxel's world position comes from the grid's index->world affine (the adjugate
recipe of nrf.index_to_world), each coordinate ((m_a0 x + m_a1 y) + m_a2 z) + m_a3 in
binary64; the voxel sets are then not boxes (gauss.render_cells tests every voxel).

exp_recipe(s) is Cody-Waite range reduction with a two-part ln 2 followed by the Taylor
series of e^r (coefficients 1/n!, n = 0..13) in Horner form, then an exact power-of-two
scaling:  k = rint(s * INV_LN2);  r = (s - k*LN2_HI) - k*LN2_LO;  p = sum c_n r^n;
result = ldexp(p, k).  LN2_HI carries 28 significant bits, so k*LN2_HI is exact.
"""
from __future__ import annotations

import numpy as np

LN2_HI = float.fromhex("0x1.62e42fe000000p-1")
LN2_LO = float.fromhex("0x1.f473de6af278fp-30")
INV_LN2 = float.fromhex("0x1.71547652b82fep+0")
# 1/n! rounded to binary64, n = 0..13
TAYLOR = [float.fromhex(h) for h in (
    "0x1.0000000000000p+0", "0x1.0000000000000p+0", "0x1.0000000000000p-1",
    "0x1.5555555555555p-3", "0x1.5555555555555p-5", "0x1.1111111111111p-7",
    "0x1.6c16c16c16c17p-10", "0x1.a01a01a01a01ap-13", "0x1.a01a01a01a01ap-16",
    "0x1.71de3a556c734p-19", "0x1.27e4fb7789f5cp-22", "0x1.ae64567f544e4p-26",
    "0x1.1eed8eff8d898p-29", "0x1.6124613a86d09p-33")]
CLAMP = float(2 ** 30)


def exp_recipe(s):
    s = np.asarray(s, dtype=np.float64)
    k = np.rint(s * INV_LN2)
    r = (s - k * LN2_HI) - k * LN2_LO
    p = np.full_like(r, TAYLOR[13])
    for n in range(12, -1, -1):
        p = p * r + TAYLOR[n]
    with np.errstate(over="ignore", under="ignore"):
        return np.ldexp(p, np.clip(k, -2000, 2000).astype(np.int64))


def rotation_recipe(wq, xq, yq, zq):
    """Rotation matrices [N,3,3] from normalised quaternion components, fixed association."""
    N = wq.shape[0]
    R = np.empty((N, 3, 3))
    R[:, 0, 0] = 1.0 - 2.0 * ((yq * yq) + (zq * zq))
    R[:, 0, 1] = 2.0 * ((xq * yq) - (wq * zq))
    R[:, 0, 2] = 2.0 * ((xq * zq) + (wq * yq))
    R[:, 1, 0] = 2.0 * ((xq * yq) + (wq * zq))
    R[:, 1, 1] = 1.0 - 2.0 * ((xq * xq) + (zq * zq))
    R[:, 1, 2] = 2.0 * ((yq * zq) - (wq * xq))
    R[:, 2, 0] = 2.0 * ((xq * zq) - (wq * yq))
    R[:, 2, 1] = 2.0 * ((yq * zq) + (wq * xq))
    R[:, 2, 2] = 1.0 - 2.0 * ((xq * xq) + (yq * yq))
    return R


def boxes(mean, quat, log_scale, logit, grid, cutoff: float = 3.0):
    """Integer boxes of every Gaussian on one grid.

    Returns (lo [N,3] int64, hi [N,3] int64, nonempty [N] bool, valid [N] bool) with
    lo/hi inclusive voxel indices (x, y, z) already clipped to the grid.
    """
    mu = np.asarray(mean, np.float32).astype(np.float64)
    q = np.asarray(quat, np.float32).astype(np.float64)
    s = np.asarray(log_scale, np.float32).astype(np.float64)
    a = np.asarray(logit, np.float32).astype(np.float64)
    L = np.asarray(grid.world_to_index, np.float64)[:, :3]
    t = np.asarray(grid.world_to_index, np.float64)[:, 3]
    sig = float(grid.psf_sigma_z)
    dims = np.array([grid.nx, grid.ny, grid.nz], dtype=np.int64)

    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    with np.errstate(invalid="ignore", over="ignore", divide="ignore"):
        n2 = ((w * w + x * x) + y * y) + z * z
        finite = (np.isfinite(mu).all(1) & np.isfinite(q).all(1) & np.isfinite(s).all(1)
                  & np.isfinite(a))
        valid = finite & (n2 > 0) & np.isfinite(n2)
        nq = np.sqrt(np.where(valid, n2, 1.0))
        R = rotation_recipe(w / nq, x / nq, y / nq, z / nq)
        e = exp_recipe(np.where(valid[:, None], s, 0.0))
        valid = valid & np.isfinite(e).all(1) & (e > 0).all(1)
        M = np.empty((mu.shape[0], 3, 3))
        for j in range(3):
            for m in range(3):
                M[:, j, m] = ((L[j, 0] * R[:, 0, m] + L[j, 1] * R[:, 1, m]) + L[j, 2] * R[:, 2, m])
        B = M * e[:, None, :]
        D = ((B[:, :, 0] * B[:, :, 0] + B[:, :, 1] * B[:, :, 1]) + B[:, :, 2] * B[:, :, 2])
        D[:, 2] = D[:, 2] + sig * sig
        rho = cutoff * np.sqrt(D)
        c = np.empty((mu.shape[0], 3))
        for j in range(3):
            c[:, j] = ((L[j, 0] * mu[:, 0] + L[j, 1] * mu[:, 1]) + L[j, 2] * mu[:, 2]) + t[j]
        lo = np.clip(np.ceil(c - rho), -CLAMP, CLAMP)
        hi = np.clip(np.floor(c + rho), -CLAMP, CLAMP)
    lo = np.where(np.isfinite(lo), lo, CLAMP).astype(np.int64)
    hi = np.where(np.isfinite(hi), hi, -CLAMP).astype(np.int64)
    lo = np.maximum(lo, 0)
    hi = np.minimum(hi, dims[None, :] - 1)
    nonempty = valid & (lo <= hi).all(1)
    return lo, hi, nonempty, valid


def world_axes(grid):
    """For an axis-aligned grid (each row of L has one non-zero entry, in distinct columns):
    the world axis of each index axis; None otherwise."""
    L = np.asarray(grid.world_to_index, np.float64)[:, :3]
    nz = [np.flatnonzero(L[j]) for j in range(3)]
    if any(len(k) != 1 for k in nz):
        return None
    axes = [int(k[0]) for k in nz]
    return axes if len(set(axes)) == 3 else None


def cell_of(x, resolution):
    """Eq. 4: cell index floor((x + 1) res / 2) along one axis, binary64, that association."""
    return np.floor(((np.asarray(x, np.float64) + 1.0) * float(resolution)) / 2.0)


def block_boxes(mean, quat, log_scale, logit, grid, resolution: int, radius: int):
    """The paper's cell-neighbourhood query (Sec. 3.3.1, Eqs. 4-6) as voxel boxes.

    [-1, 1]^3 is cut into resolution^3 cells; voxel v of the grid takes Gaussian i when, on
    every world axis a, |cell_a(x(v)) - cell_a(mu_i)| <= radius (Eqs. 5-6).  On an axis-aligned
    grid the world coordinate of v along world axis a depends on one index axis j only:
    x_a = (v_j - t_j) / L[j, a] (binary64), so the voxels form a box.  Gaussians whose
    parameters are invalid (as in boxes()) get none.  Returns (lo, hi, nonempty, valid) like
    boxes()."""
    axes = world_axes(grid)
    if axes is None:
        raise ValueError("the block query needs an axis-aligned grid")
    _, _, _, valid = boxes(mean, quat, log_scale, logit, grid)
    mu = np.asarray(mean, np.float32).astype(np.float64)
    A = np.asarray(grid.world_to_index, np.float64)
    dims = [grid.nx, grid.ny, grid.nz]
    n = mu.shape[0]
    lo = np.zeros((n, 3), np.int64)
    hi = np.zeros((n, 3), np.int64)
    nonempty = valid.copy()
    for j in range(3):
        a = axes[j]
        v = np.arange(dims[j], dtype=np.float64)
        cells = cell_of((v - A[j, 3]) / A[j, a], resolution)     # monotone in v
        with np.errstate(invalid="ignore"):
            cm = cell_of(np.where(valid, mu[:, a], 0.0), resolution)
        if A[j, a] > 0:
            first = np.searchsorted(cells, cm - radius, side="left")
            last = np.searchsorted(cells, cm + radius, side="right") - 1
        else:
            rc = cells[::-1]
            first = dims[j] - np.searchsorted(rc, cm + radius, side="right")
            last = dims[j] - 1 - np.searchsorted(rc, cm - radius, side="left")
        lo[:, j], hi[:, j] = first, last
        nonempty &= first <= last
    return lo, hi, nonempty, valid


def voxel_cells(grid, resolution: int):
    """Eq. 4 cell, per world axis, of every voxel's world position: [n_voxels, 3] int64 in
    storage order ([z][y][x]).  x_a = ((M_a0 x + M_a1 y) + M_a2 z) + M_a3 (binary64) with
    M = the grid's index->world affine by the adjugate recipe."""
    from .nrf import index_to_world
    M = index_to_world(grid.world_to_index)
    z, y, x = np.meshgrid(np.arange(grid.nz, dtype=np.float64),
                          np.arange(grid.ny, dtype=np.float64),
                          np.arange(grid.nx, dtype=np.float64), indexing="ij")
    x, y, z = x.reshape(-1), y.reshape(-1), z.reshape(-1)
    out = np.empty((x.shape[0], 3), np.int64)
    for a in range(3):
        w = ((M[a, 0] * x + M[a, 1] * y) + M[a, 2] * z) + M[a, 3]
        out[:, a] = cell_of(w, resolution).astype(np.int64)
    return out


def mean_cells(mean, resolution: int):
    """Eq. 4 cell of each Gaussian's mean (float32 inputs in binary64), clamped to
    [-2^30, 2^30] (no voxel of a grid of at most 32768 voxels a side within world
    coordinates of magnitude 1000 has a cell beyond 2^30 - 2^21 at resolutions up to 2^20, so
    the clamp changes no comparison); 0 where not finite (such Gaussians are invalid and take
    no voxel)."""
    mu = np.asarray(mean, np.float32).astype(np.float64)
    with np.errstate(invalid="ignore", over="ignore"):
        c = cell_of(np.where(np.isfinite(mu), mu, 0.0), resolution)
    return np.clip(c, -2.0 ** 30, 2.0 ** 30).astype(np.int64)


def box_volume(lo, hi, nonempty):
    v = np.prod(hi - lo + 1, axis=1)
    return np.where(nonempty, v, 0)


def tile_counts(lo, hi, nonempty, tile):
    """Tiles each box overlaps, for tile edge lengths tile = (TX, TY, TZ)."""
    T = np.asarray(tile, dtype=np.int64)
    span = hi // T - lo // T + 1
    return np.where(nonempty, np.prod(span, axis=1), 0)


def tile_lists(lo, hi, nonempty, grid, tile, base: int = 0):
    """Per-tile lists, ascending Gaussian id, as (tile_ids, gauss_ids) pairs sorted by
    (tile, gauss) - brute force over every box's tile range."""
    T = np.asarray(tile, dtype=np.int64)
    ntx = -(-grid.nx // T[0])
    nty = -(-grid.ny // T[1])
    tiles, gids = [], []
    for i in np.nonzero(nonempty)[0]:
        t0 = lo[i] // T
        t1 = hi[i] // T
        for tz in range(t0[2], t1[2] + 1):
            for ty in range(t0[1], t1[1] + 1):
                for tx in range(t0[0], t1[0] + 1):
                    tiles.append(base + (tz * nty + ty) * ntx + tx)
                    gids.append(i)
    tiles = np.asarray(tiles, dtype=np.int64)
    gids = np.asarray(gids, dtype=np.int64)
    order = np.lexsort((gids, tiles))
    return tiles[order], gids[order]


def n_tiles(grid, tile):
    T = np.asarray(tile, dtype=np.int64)
    return int((-(-grid.nx // T[0])) * (-(-grid.ny // T[1])) * (-(-grid.nz // T[2])))


def csr_from_pairs(tiles, gids, total_tiles):
    counts = np.bincount(tiles, minlength=total_tiles)
    start = np.zeros(total_tiles + 1, dtype=np.int64)
    np.cumsum(counts, out=start[1:])
    return start, gids

"""Seeded synthetic inputs: phantoms, thick-slice stacks, grid descriptors, Gaussian inits.

This module is the only code shared by the GPU path's tests and the CPU oracle's tests.
It holds no Gaussian-evaluation arithmetic: it builds ground-truth volumes, simulates
thick-slice acquisitions of them, describes voxel grids as affine maps and draws random
Gaussian parameters.  Everything is seeded through numpy's PCG64.

Conventions (the paper normalises space to [-1, 1]^3, Sec. 3.1 and Eq. 2):
  * A grid of n voxels along an axis is cell-centred: voxel i has world coordinate
    -1 + (2 i + 1) / n, so index = (x + 1) n / 2 - 1/2.
  * Arrays are stored [nz][ny][nx], x fastest.  A stack's index z is its slice number.
  * A grid maps world -> index through a 3x4 affine A = [L | t] (float64, row-major).
  * Stacks carry a Gaussian slice profile along their index z (the slice normal):
    FWHM = slice thickness, i.e. sigma = FWHM / (2 sqrt(2 ln 2)) in slice units.
  * Gaussian parameters: mean [N,3] world coords, quat [N,4] (w,x,y,z, unnormalised),
    log_scale [N,3] (log of the world-space standard deviations), logit [N]
    (intensity alpha = sigmoid(logit)).  All float32.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


@dataclasses.dataclass(frozen=True)
class Grid:
    """A voxel grid: dims (nx, ny, nz), world->index affine (3x4), slice-profile sigma."""
    nx: int
    ny: int
    nz: int
    world_to_index: np.ndarray  # (3, 4) float64
    psf_sigma_z: float = 0.0    # std-dev of the slice profile along index z, in index units
    name: str = ""

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz

    def index_to_world(self) -> np.ndarray:
        L = self.world_to_index[:, :3]
        t = self.world_to_index[:, 3]
        Li = np.linalg.inv(L)
        return np.concatenate([Li, (-Li @ t)[:, None]], axis=1)


@dataclasses.dataclass
class Gaussians:
    mean: np.ndarray       # [N,3] f32
    quat: np.ndarray       # [N,4] f32
    log_scale: np.ndarray  # [N,3] f32
    logit: np.ndarray      # [N]   f32

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    def subset(self, idx) -> "Gaussians":
        return Gaussians(self.mean[idx].copy(), self.quat[idx].copy(),
                         self.log_scale[idx].copy(), self.logit[idx].copy())


# ----------------------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------------------

def _axis_map(n: int):
    """world -> index along one axis for a cell-centred grid of n voxels over [-1, 1]."""
    return n / 2.0, n / 2.0 - 0.5


def volume_grid(n: int, name: str = "volume") -> Grid:
    s, o = _axis_map(n)
    A = np.zeros((3, 4))
    A[0, 0] = A[1, 1] = A[2, 2] = s
    A[:, 3] = o
    return Grid(n, n, n, A, 0.0, name)


def _rotation_axis_angle(axis: np.ndarray, angle: float) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


# stack index axis (x_s, y_s, z_s) -> world axis; z_s is the slice normal
_ORIENT = {
    "axial": (0, 1, 2),
    "coronal": (0, 2, 1),
    "sagittal": (1, 2, 0),
}


def stack_grid(orient: str, n_inplane: int, n_slices: int, fwhm_slices: float = 1.0,
               rigid: Optional[np.ndarray] = None, shift: Optional[np.ndarray] = None,
               name: str = "") -> Grid:
    """A thick-slice stack over [-1,1]^3.

    n_inplane voxels along the two in-plane axes, n_slices along the normal.  The slice
    profile has FWHM ``fwhm_slices`` slice spacings.  ``rigid`` (3x3 rotation about the
    volume centre) and ``shift`` (world units) place the stack: the stack voxel at index v
    samples the world point T(P(v)) with P the nominal index->world map and T(x) = R x + s.
    """
    perm = _ORIENT[orient]
    dims = (n_inplane, n_inplane, n_slices)
    P = np.zeros((3, 3))       # nominal world->index linear part
    t = np.zeros(3)
    for k in range(3):
        s, o = _axis_map(dims[k])
        P[k, perm[k]] = s
        t[k] = o
    R = np.eye(3) if rigid is None else np.asarray(rigid, dtype=np.float64)
    sh = np.zeros(3) if shift is None else np.asarray(shift, dtype=np.float64)
    # index = P (R^T (x - sh)) + t
    L = P @ R.T
    A = np.concatenate([L, (t - L @ sh)[:, None]], axis=1)
    return Grid(dims[0], dims[1], dims[2], A, float(fwhm_slices) * FWHM_TO_SIGMA,
                name or orient)


def random_rigid(rng: np.random.Generator, max_deg: float, max_shift_vox: float, n: int):
    """Rotation about a uniformly random axis by U(-max_deg, max_deg) degrees and a shift of
    U(-max_shift_vox, max_shift_vox) voxels (of an n-voxel volume) per axis."""
    axis = rng.normal(size=3)
    ang = math.radians(rng.uniform(-max_deg, max_deg))
    R = _rotation_axis_angle(axis, ang)
    shift = rng.uniform(-max_shift_vox, max_shift_vox, size=3) * (2.0 / n)
    return R, shift


# ----------------------------------------------------------------------------------------
# phantoms and simulated acquisitions
# ----------------------------------------------------------------------------------------

def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def make_phantom(n: int, n_ellipsoids: int, rng: np.random.Generator, bias: bool = False,
                 noise: float = 0.0, device="cpu"):
    """Piecewise-constant ellipsoid phantom on an n^3 cell-centred grid, values in [0, 1].

    Centres U[-0.6,0.6]^3, semi-axes U[0.08,0.45], uniform random orientation, intensity
    U(0.2, 1), composited by maximum over a zero background.  With ``bias`` the volume is
    multiplied by a smooth field exp(sum of degree 1..2 monomials, coefficients N(0, 0.1^2)).
    Random draws come from ``rng``; the voxel arithmetic runs in torch on ``device``.
    Returns a float32 torch tensor [n, n, n] on ``device``.
    """
    import torch
    dev = torch.device(device)
    coords = (-1.0 + (2.0 * torch.arange(n, device=dev, dtype=torch.float32) + 1.0) / n)
    vol = torch.zeros((n, n, n), dtype=torch.float32, device=dev)
    cnp = coords.cpu().numpy()
    for _ in range(n_ellipsoids):
        c = rng.uniform(-0.6, 0.6, size=3)
        ax = rng.uniform(0.08, 0.45, size=3)
        R = _random_rotation(rng)
        val = float(rng.uniform(0.2, 1.0))
        r = float(ax.max())
        lo = np.searchsorted(cnp, c - r, side="left")
        hi = np.searchsorted(cnp, c + r, side="right")
        if np.any(hi <= lo):
            continue
        zs, ys, xs = (coords[lo[2]:hi[2]], coords[lo[1]:hi[1]], coords[lo[0]:hi[0]])
        Z, Y, X = torch.meshgrid(zs, ys, xs, indexing="ij")
        Rt = torch.tensor(R, dtype=torch.float32, device=dev)
        P = torch.stack([X - float(c[0]), Y - float(c[1]), Z - float(c[2])], dim=-1) @ Rt
        axt = torch.tensor(ax, dtype=torch.float32, device=dev)
        inside = ((P / axt) ** 2).sum(-1) <= 1.0
        sub = vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        torch.maximum(sub, inside.to(torch.float32) * val, out=sub)
    if bias:
        Z, Y, X = torch.meshgrid(coords, coords, coords, indexing="ij")
        mons = [X, Y, Z, X * X, Y * Y, Z * Z, X * Y, X * Z, Y * Z]
        coef = rng.normal(0.0, 0.1, size=len(mons))
        field = torch.exp(sum(float(cf) * m for cf, m in zip(coef, mons)))
        vol = torch.clamp(vol * field, 0.0, 1.0)
    if noise > 0:
        vol = vol + torch.from_numpy(rng.normal(0.0, noise, size=vol.shape).astype(np.float32)).to(dev)
    return vol.contiguous()


def slice_grids(stack: Grid) -> List[Grid]:
    """The stack's slices as one-slice grids: slice k keeps the stack's in-plane indexing and
    slice profile, and its index z is the stack's minus k (so the slice sits at z = 0).  With
    the stack's placement they give the stack's values slice by slice; each can then carry its
    own rigid transform T_k (Sec. 3.3.2: every slice is moved by its own T_k)."""
    out = []
    A = np.asarray(stack.world_to_index, np.float64)
    for k in range(stack.nz):
        Ak = A.copy()
        Ak[2, 3] -= k
        out.append(Grid(stack.nx, stack.ny, 1, Ak, stack.psf_sigma_z, f"{stack.name}[{k}]"))
    return out


def simulate_stack(vol, grid: Grid, rng: np.random.Generator, noise: float = 0.01,
                   samples_per_slice: int = 8):
    """Acquire a thick-slice stack of the cell-centred volume ``vol`` (torch [n,n,n]).

    Each stack voxel integrates the volume along the slice normal with the grid's Gaussian
    slice profile (supersampled ``samples_per_slice`` per slice spacing over +-3 sigma) and
    point-samples in-plane by trilinear interpolation (zero outside the volume); then
    N(0, noise^2) is added.  Runs in torch on vol's device; returns a float32 tensor
    [nz, ny, nx] on that device.
    """
    import torch
    import torch.nn.functional as F
    dev = vol.device
    Ainv = torch.tensor(grid.index_to_world(), dtype=torch.float64, device=dev)
    sig = grid.psf_sigma_z
    if sig > 0:
        half = 3.0 * sig
        m = max(1, int(math.ceil(2 * half * samples_per_slice)))
        us = np.linspace(-half, half, m + 1)
        ws = np.exp(-0.5 * (us / sig) ** 2)
        ws /= ws.sum()
    else:
        us, ws = np.array([0.0]), np.array([1.0])
    out = torch.zeros(grid.shape, dtype=torch.float64, device=dev)
    zz, yy, xx = torch.meshgrid(torch.arange(grid.nz, device=dev, dtype=torch.float64),
                                torch.arange(grid.ny, device=dev, dtype=torch.float64),
                                torch.arange(grid.nx, device=dev, dtype=torch.float64),
                                indexing="ij")
    v5 = vol[None, None]
    for u, w in zip(us, ws):
        p = torch.stack([xx, yy, zz + float(u)], dim=-1)
        world = p @ Ainv[:, :3].T + Ainv[:, 3]
        # grid_sample with align_corners=False addresses voxel centres at -1 + (2i+1)/n,
        # the same cell-centred convention as the world frame here
        smp = F.grid_sample(v5, world.to(torch.float32)[None], mode="bilinear",
                            padding_mode="zeros", align_corners=False)[0, 0]
        out += float(w) * smp.to(torch.float64)
    if noise > 0:
        out += torch.from_numpy(rng.normal(0.0, noise, size=grid.shape)).to(dev)
    return out.to(torch.float32).contiguous()


# ----------------------------------------------------------------------------------------
# Gaussian initialisations
# ----------------------------------------------------------------------------------------

def random_voxel_centres(n_vox: int, count: int, rng: np.random.Generator,
                         jitter: bool = False) -> np.ndarray:
    flat = rng.choice(n_vox ** 3, size=count, replace=False)
    iz, rem = np.divmod(flat, n_vox * n_vox)
    iy, ix = np.divmod(rem, n_vox)
    idx = np.stack([ix, iy, iz], axis=1).astype(np.float64)
    if jitter:
        idx += rng.uniform(-0.5, 0.5, size=idx.shape)
    return (-1.0 + (2.0 * idx + 1.0) / n_vox).astype(np.float32)


def init_isotropic(n_vox: int, count: int, rng: np.random.Generator,
                   sigma_vox: float = 1.0) -> Gaussians:
    """Distinct random voxel centres, isotropic sigma_vox voxels, identity rotation,
    logit ~ N(0, 1)."""
    mean = random_voxel_centres(n_vox, count, rng)
    quat = np.zeros((count, 4), np.float32)
    quat[:, 0] = 1.0
    ls = np.full((count, 3), math.log(sigma_vox * 2.0 / n_vox), np.float32)
    logit = rng.normal(0.0, 1.0, size=count).astype(np.float32)
    return Gaussians(mean, quat, ls, logit)


def init_anisotropic(n_vox: int, count: int, rng: np.random.Generator,
                     log_sd: float = 0.3, jitter: bool = True) -> Gaussians:
    """Random voxel centres (jittered within the voxel), log-scales ln(2/n) + N(0, log_sd^2)
    (one voxel on average), uniformly random unit quaternions, logit ~ N(0, 1)."""
    mean = random_voxel_centres(n_vox, count, rng, jitter=jitter)
    q = rng.normal(size=(count, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    ls = (math.log(2.0 / n_vox) + rng.normal(0.0, log_sd, size=(count, 3)))
    logit = rng.normal(0.0, 1.0, size=count)
    return Gaussians(mean, q.astype(np.float32), ls.astype(np.float32),
                     logit.astype(np.float32))


# ----------------------------------------------------------------------------------------
# workload configurations
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    n_vox: int
    stacks: List[Grid]
    volume: Grid
    gauss: Gaussians
    phantom: Optional[object] = None     # [n,n,n] float32 (numpy on cpu, else torch)
    stack_data: Optional[List[object]] = None


def orthogonal_stacks(n: int, n_slices: int, fwhm_slices: float, rng=None,
                      rigid_deg: float = 0.0, rigid_shift: float = 0.0) -> List[Grid]:
    out = []
    for o in ("axial", "coronal", "sagittal"):
        R = sh = None
        if rng is not None and (rigid_deg > 0 or rigid_shift > 0):
            R, sh = random_rigid(rng, rigid_deg, rigid_shift, n)
        out.append(stack_grid(o, n, n_slices, fwhm_slices, R, sh))
    return out


def oblique_stacks(n: int, n_slices: int, fwhm_slices: float, deg: float = 30.0) -> List[Grid]:
    """The axial stack tilted by ``deg`` about world x, and by ``deg`` about world y."""
    a = math.radians(deg)
    return [stack_grid("axial", n, n_slices, fwhm_slices,
                       _rotation_axis_angle([1, 0, 0], a), None, "oblique_x"),
            stack_grid("axial", n, n_slices, fwhm_slices,
                       _rotation_axis_angle([0, 1, 0], a), None, "oblique_y")]


def workload(name: str, with_data: bool = True, seed: Optional[int] = None,
             device="cpu") -> Workload:
    """The synthetic workloads.

    (Gaussians in raster order of their voxel, as a devoxelised lattice stores them)
    small     : 24^3 volume, 3 stacks 24x24x6, 300 anisotropic Gaussians (fast tests)
    c64       : 64^3, 12 ellipsoids, 3 x 64x64x16, FWHM 4 voxels, 20k isotropic 1-voxel
                Gaussians at distinct voxel centres
    c128      : 128^3, 40 ellipsoids x bias, 3 x 128x128x32 with +-2 deg / +-1 voxel rigid
                offsets, 200k anisotropic Gaussians
    c256      : 256^3, 120 ellipsoids, 3 x 256x256x64 (rigid offsets as c128), 1M
                anisotropic Gaussians
    c320      : 320^3, 3 orthogonal + 2 oblique (30 deg) stacks of 320x320x80, slice
                thickness 5 voxels at spacing 4, 2M anisotropic Gaussians
    """
    cfg = {
        "small": dict(n=24, ell=4, sl=6, fw=1.0, ng=300, iso=False, rig=(2.0, 1.0), bias=False, seed=11),
        "c64": dict(n=64, ell=12, sl=16, fw=1.0, ng=20_000, iso=True, rig=(0.0, 0.0), bias=False, seed=1001),
        "c128": dict(n=128, ell=40, sl=32, fw=1.0, ng=200_000, iso=False, rig=(2.0, 1.0), bias=True, seed=2001),
        "c256": dict(n=256, ell=120, sl=64, fw=1.0, ng=1_000_000, iso=False, rig=(2.0, 1.0), bias=False, seed=3001),
        "c320": dict(n=320, ell=150, sl=80, fw=1.25, ng=2_000_000, iso=False, rig=(0.0, 0.0), bias=False, seed=5001),
    }[name]
    ss = np.random.SeedSequence(cfg["seed"] if seed is None else seed)
    r_ph, r_st, r_noise, r_init = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(4)]
    n = cfg["n"]
    stacks = orthogonal_stacks(n, cfg["sl"], cfg["fw"], r_st, *cfg["rig"])
    if name == "c320":
        stacks += oblique_stacks(n, cfg["sl"], cfg["fw"])
    vol = volume_grid(n)
    if cfg["iso"]:
        g = init_isotropic(n, cfg["ng"], r_init)
    else:
        g = init_anisotropic(n, cfg["ng"], r_init)
    # stored in raster order of their voxel, as a devoxelised lattice stores its Gaussians
    g = g.subset(raster_order(g.mean, n))
    w = Workload(name, n, stacks, vol, g)
    if with_data:
        w.phantom = make_phantom(n, cfg["ell"], r_ph, bias=cfg["bias"], device=device)
        w.stack_data = [simulate_stack(w.phantom, s, r_noise, 0.01) for s in stacks]
        if str(device) == "cpu":
            w.phantom = w.phantom.numpy()
            w.stack_data = [d.numpy() for d in w.stack_data]
    return w


def raster_order(mean: np.ndarray, n: int) -> np.ndarray:
    """Permutation that sorts Gaussians by the voxel of an n^3 grid over [-1, 1]^3 holding
    their mean, x fastest (stable)."""
    v = np.floor((np.asarray(mean, np.float64) + 1.0) * n / 2.0).astype(np.int64).clip(0, n - 1)
    return np.argsort((v[:, 2] * n + v[:, 1]) * n + v[:, 0], kind="stable")


def random_dl_di(grids: Sequence[Grid], rng: np.random.Generator, scale: float = 1.0):
    """Seeded per-voxel upstream gradients dL/dI for each grid (float32)."""
    return [(rng.normal(size=g.shape) * scale).astype(np.float32) for g in grids]


def slice_pair(shape, rng: np.random.Generator):
    """Seeded (prediction, target) float32 stacks [nz, ny, nx] for the SSIM term.  Each target
    slice holds 6 random ellipses, piecewise constant with values U(0.2, 1) over a zero
    background, plus noise N(0, 0.01^2); the prediction is the target averaged over 3 x 3
    in-plane neighbours (edge-replicated), scaled by 0.95, plus noise N(0, 0.005^2)."""
    nz, ny, nx = shape
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    tgt = np.zeros(shape)
    for z in range(nz):
        for _ in range(6):
            cy, cx = rng.uniform(0, ny), rng.uniform(0, nx)
            ry, rx = rng.uniform(0.1, 0.5) * ny + 1, rng.uniform(0.1, 0.5) * nx + 1
            tgt[z][((yy - cy) / ry) ** 2 + ((xx - cx) / rx) ** 2 <= 1.0] = rng.uniform(0.2, 1.0)
    tgt += rng.normal(0.0, 0.01, size=shape)
    pad = np.pad(tgt, ((0, 0), (1, 1), (1, 1)), mode="edge")
    avg = sum(pad[:, i:i + ny, j:j + nx] for i in range(3) for j in range(3)) / 9.0
    pred = 0.95 * avg + rng.normal(0.0, 0.005, size=shape)
    return pred.astype(np.float32), tgt.astype(np.float32)

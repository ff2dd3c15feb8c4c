"""Joint optimisation of the stacks' rigid transforms T_k (Sec. 3.3.2): host-side chain from
the library's affine gradient (gm_grid_pose_grads) to a rigid increment, and its Adam step.

A stack grid's world->index affine is A = [L | t] with v = L x + t.  The stack was placed by a
rigid motion T(x_s) = R x_s + tau from its own frame into the volume, so with the nominal
affine A0 = [L0 | t0] (T = identity)
    L = L0 R^T,   t = t0 - L0 R^T tau.
The pose is updated on the rotation group: R <- exp([d_omega]x) R, tau <- tau + d_tau.  For the
objective's gradient G = [G_L | G_t] = dObj/dA at the current pose, the gradient with respect to
the increment (d_omega, d_tau) at zero is
    d_tau:   -R L0^T G_t
    d_omega: vee of the skew part of Q = -R L0^T (G_L - G_t tau^T), i.e.
             (Q32 - Q23, Q13 - Q31, Q21 - Q12)   (1-based indices)
since dA = [-L0 R^T [d_omega]x | L0 R^T [d_omega]x tau - L0 R^T d_tau].  A pose may instead
rotate about its own centre c (a slice's centre, where its rotation and translation decouple):
T(x_s) = R (x_s - c) + c + tau is the origin form with tau' = tau + c - R c, and under the same
increment tau' moves by d_tau - [d_omega]x R c, so d_omega's gradient gains - (R c) x g_tau'.
This module is 6 numbers per stack (or slice) of host arithmetic; every voxel-level step runs
in the library.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import inputs


def skew(w) -> np.ndarray:
    w = np.asarray(w, np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def rotvec_to_matrix(w) -> np.ndarray:
    """exp([w]x) by Rodrigues' formula (series for tiny angles)."""
    w = np.asarray(w, np.float64)
    th = float(np.linalg.norm(w))
    K = skew(w)
    if th < 1e-8:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + (np.sin(th) / th) * K + ((1.0 - np.cos(th)) / (th * th)) * K @ K


def grid_centre(grid: inputs.Grid) -> np.ndarray:
    """World coordinates of the centre of a grid's voxel lattice (index ((n - 1) / 2) per
    axis)."""
    M = grid.index_to_world()
    v = np.array([(grid.nx - 1) / 2.0, (grid.ny - 1) / 2.0, (grid.nz - 1) / 2.0])
    return M[:, :3] @ v + M[:, 3]


@dataclasses.dataclass
class StackPose:
    """Pose of one stack (or slice): nominal grid (T = identity) and the current rigid motion,
    rotating about the world origin, or about `centre` (world coordinates) when it is given."""
    nominal: inputs.Grid
    R: np.ndarray = dataclasses.field(default_factory=lambda: np.eye(3))
    tau: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    centre: Optional[np.ndarray] = None

    def tau_origin(self) -> np.ndarray:
        """The translation of the same motion written as a rotation about the origin."""
        if self.centre is None:
            return self.tau
        c = np.asarray(self.centre, np.float64)
        return self.tau + c - self.R @ c

    def affine(self) -> np.ndarray:
        A0 = np.asarray(self.nominal.world_to_index, np.float64)
        L0, t0 = A0[:, :3], A0[:, 3]
        L = L0 @ self.R.T
        return np.concatenate([L, (t0 - L @ self.tau_origin())[:, None]], axis=1)

    def grid(self) -> inputs.Grid:
        g = self.nominal
        return inputs.Grid(g.nx, g.ny, g.nz, self.affine(), g.psf_sigma_z, g.name)

    def tangent_grad(self, G) -> np.ndarray:
        """(d_omega, d_tau) gradient [6] from dObj/dA (3x4) at the current pose."""
        G = np.asarray(G, np.float64)
        G_L, G_t = G[:, :3], G[:, 3]
        L0 = np.asarray(self.nominal.world_to_index, np.float64)[:, :3]
        Q = -self.R @ L0.T @ (G_L - np.outer(G_t, self.tau_origin()))
        g_w = np.array([Q[2, 1] - Q[1, 2], Q[0, 2] - Q[2, 0], Q[1, 0] - Q[0, 1]])
        g_t = -self.R @ L0.T @ G_t
        if self.centre is not None:
            g_w = g_w - np.cross(self.R @ np.asarray(self.centre, np.float64), g_t)
        return np.concatenate([g_w, g_t])

    def apply(self, d) -> None:
        """R <- exp([d_omega]x) R, tau <- tau + d_tau."""
        d = np.asarray(d, np.float64)
        self.R = rotvec_to_matrix(d[:3]) @ self.R
        self.tau = self.tau + d[3:]


class PoseAdam:
    """Adam on the rigid increments of several stacks (moments in the tangent space of each
    pose, FP64 on the host): learning rates for rotation (radians) and translation (world
    units, [-1, 1]^3)."""

    def __init__(self, poses: Sequence[StackPose], lr_rot: float = 1e-3, lr_trans: float = 1e-3,
                 beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                 frozen: Sequence[int] = ()):
        self.poses = list(poses)
        self.lr = np.array([lr_rot] * 3 + [lr_trans] * 3)
        self.b1, self.b2, self.eps = beta1, beta2, eps
        self.m = [np.zeros(6) for _ in self.poses]
        self.v = [np.zeros(6) for _ in self.poses]
        self.frozen = set(frozen)   # e.g. a reference stack that fixes the gauge
        self.t = 0

    def step(self, affine_grads: Sequence[np.ndarray]) -> List[np.ndarray]:
        self.t += 1
        bc1, bc2 = 1 - self.b1 ** self.t, 1 - self.b2 ** self.t
        steps = []
        for k, (pose, G) in enumerate(zip(self.poses, affine_grads)):
            if k in self.frozen:
                steps.append(np.zeros(6))
                continue
            g = pose.tangent_grad(G)
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g * g
            d = -self.lr / bc1 * self.m[k] / (np.sqrt(self.v[k]) / np.sqrt(bc2) + self.eps)
            pose.apply(d)
            steps.append(d)
        return steps

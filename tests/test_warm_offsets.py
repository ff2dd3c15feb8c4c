"""The control arm's constant offsets (closed forms in warmstart.constant_offsets) against a
direct minimisation of the same loss over a fine grid of offsets."""
import numpy as np
import torch

from paper_2603_00145_amd import warmstart


def test_constant_offsets_minimise_the_loss():
    rng = np.random.default_rng(3)
    n = 4000
    s0 = np.full((n, 3), np.log(0.02))
    l0 = rng.normal(0.0, 0.5, n)
    # targets: random rotations of anisotropic scales around the initial one
    s_t = np.log(0.02) + rng.normal(0.3, 0.4, (n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                  2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                  2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1).reshape(n, 3, 3)
    Sig = R @ (np.exp(2 * s_t)[:, :, None] * np.transpose(R, (0, 2, 1)))
    sig6 = np.stack([Sig[:, 0, 0], Sig[:, 1, 1], Sig[:, 2, 2], Sig[:, 0, 1], Sig[:, 0, 2],
                     Sig[:, 1, 2]], 1)
    lt = l0 + rng.normal(0.7, 0.3, n)
    T = lambda a: torch.from_numpy(np.asarray(a))
    d, e = warmstart.constant_offsets(T(s0), T(l0), T(sig6), T(lt))
    nrm = (Sig ** 2).sum((1, 2))

    def loss(dd):
        u = np.exp(2 * (s0[:, 0] + dd))
        return np.mean(((u[:, None, None] * np.eye(3) - Sig) ** 2).sum((1, 2)) / nrm)

    grid = d + np.linspace(-0.5, 0.5, 2001)
    vals = [loss(g) for g in grid]
    assert abs(grid[int(np.argmin(vals))] - d) <= 1e-3
    assert loss(d) <= min(vals) + 1e-12
    lg = np.linspace(e - 0.5, e + 0.5, 2001)
    lv = [np.mean((l0 + g - lt) ** 2) for g in lg]
    assert abs(lg[int(np.argmin(lv))] - e) <= 1e-3

"""Pins of the oracle's warm-start network: conv layers and their gradients against torch
float64 (an independent implementation), the loss gradient against central differences, and
the patch gather against direct sampling."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import warm
from paper_2603_00145_amd import inputs


def rand_net(rng):
    net = {}
    for l, (ci, co, k, st, pd, di, do) in enumerate(warm.LAYERS):
        net[f"W{l + 1}"] = rng.normal(0, 0.3, (co, ci, k, k, k))
        net[f"b{l + 1}"] = rng.normal(0, 0.1, co)
    net["Wl"] = rng.normal(0, 0.3, (8, 32))
    net["bl"] = rng.normal(0, 0.1, 8)
    return net


def torch_forward(net, X0):
    a = torch.from_numpy(X0)
    ws = {k: torch.from_numpy(v).requires_grad_(True) for k, v in net.items()}
    for l, (ci, co, k, st, pd, di, do) in enumerate(warm.LAYERS):
        a = F.silu(F.conv3d(a, ws[f"W{l + 1}"], ws[f"b{l + 1}"], stride=st, padding=pd))
    out = a.reshape(a.shape[0], 32) @ ws["Wl"].T + ws["bl"]
    return out, ws


def test_forward_and_backward_match_torch_float64():
    rng = np.random.default_rng(0)
    net = rand_net(rng)
    X0 = rng.normal(size=(5, 3, 8, 8, 8))
    out, _, _ = warm.forward(net, X0)
    tout, ws = torch_forward(net, X0)
    assert np.allclose(out, tout.detach().numpy(), rtol=1e-12, atol=1e-12)
    dout = rng.normal(size=out.shape)
    g = warm.backward(net, X0, dout)
    (tout * torch.from_numpy(dout)).sum().backward()
    for k in net:
        assert np.allclose(g[k], ws[k].grad.numpy(), rtol=1e-10, atol=1e-11), k


def test_loss_gradient_central_differences():
    rng = np.random.default_rng(1)
    B = 6
    out = rng.normal(0, 0.3, (B, 8))
    s0 = rng.normal(-3, 0.2, (B, 3))
    lg0 = rng.normal(size=B)
    s_t = rng.normal(-3, 0.3, (B, 3))
    q_t = rng.normal(size=(B, 4))
    sig_t = warm.covariance(s_t, q_t)
    lg_t = rng.normal(size=B)
    L, d = warm.loss_grad(out, s0, lg0, sig_t, lg_t)
    assert L == pytest.approx(warm.loss(out, s0, lg0, sig_t, lg_t), rel=1e-14)
    for i in range(B):
        for j in range(8):
            h = 1e-6
            op, om = out.copy(), out.copy()
            op[i, j] += h
            om[i, j] -= h
            fd = (warm.loss(op, s0, lg0, sig_t, lg_t) - warm.loss(om, s0, lg0, sig_t, lg_t)) / (2 * h)
            assert d[i, j] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_gather_constant_and_ramp():
    n = 16
    stacks = inputs.orthogonal_stacks(n, 4, 1.0)
    data = [np.full(s.shape, 0.5, np.float32) for s in stacks]
    X = warm.gather(stacks, data, np.zeros((1, 3)), 2.0 / n)
    assert np.allclose(X, 0.5)
    # far outside every stack: zeros
    X = warm.gather(stacks, data, np.array([[5.0, 5.0, 5.0]]), 2.0 / n)
    assert np.all(X == 0)

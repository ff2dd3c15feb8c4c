"""Pins of the oracle's neural residual field (CPU only)."""
import math

import numpy as np
import pytest
import torch

from oracle import nrf
from paper_2603_00145_amd import inputs


def random_weights(rng, in_pad, in_dim, depth, width=64):
    def bf(a):
        return nrf.bf16_round(a.astype(np.float32)).astype(np.float64)
    W0 = np.zeros((width, in_pad))
    W0[:, :in_dim] = bf(rng.uniform(-0.3, 0.3, (width, in_dim)))
    Ws = [W0] + [bf(rng.uniform(-0.2, 0.2, (width, width))) for _ in range(depth - 1)]
    bs = [rng.uniform(-0.1, 0.1, width) for _ in range(depth)]
    return {"W": Ws, "b": bs, "w_out": bf(rng.uniform(-0.3, 0.3, width)), "b_out": 0.05}


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    a = np.concatenate([(rng.normal(size=10000) * 10.0 ** rng.integers(-8, 8, 10000)).astype(np.float32),
                        np.array([1.0, -2.5, 3.0078125, 1 + 2 ** -8, 1 + 3 * 2 ** -9], np.float32)])
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(nrf.bf16_round(a), ref)


def test_encoding_matches_direct_formula():
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, (500, 3)).astype(np.float32)
    f = nrf.encode(x, 10, 64)
    xd = x.astype(np.float64)
    assert np.array_equal(f[:, :3], xd)
    for k in range(10):
        assert np.allclose(f[:, 3 + 6 * k:6 + 6 * k], np.sin(2 ** k * np.pi * xd), atol=1e-9)
        assert np.allclose(f[:, 6 + 6 * k:9 + 6 * k], np.cos(2 ** k * np.pi * xd), atol=1e-9)
    assert np.all(f[:, 63:] == 0)


def test_world_coords_cell_centres():
    g = inputs.volume_grid(20)
    M = g.index_to_world()
    vox = np.array([[0, 0, 0], [19, 7, 3], [10, 10, 10]])
    x = nrf.world_coords(vox, M)
    assert np.allclose(x, -1 + (2 * vox + 1) / 20, atol=1e-7)


@pytest.mark.parametrize("depth,n_freq,in_pad", [(3, 16, 128), (4, 6, 64)])
def test_forward_backward_match_torch_float64(depth, n_freq, in_pad):
    rng = np.random.default_rng(depth)
    w = random_weights(rng, in_pad, 3 + 6 * n_freq, depth)
    x = rng.uniform(-1, 1, (64, 3)).astype(np.float32)
    feats = nrf.encode(x, n_freq, in_pad)
    dl = rng.normal(size=64)
    r, *_ = nrf.forward(w, feats)
    g = nrf.backward(w, feats, dl)
    # independent torch float64 module with the same weights
    layers = []
    tw = []
    for Wl, bl in zip(w["W"], w["b"]):
        lin = torch.nn.Linear(Wl.shape[1], Wl.shape[0], dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(Wl))
            lin.bias.copy_(torch.from_numpy(bl))
        layers += [lin, torch.nn.SiLU()]
        tw.append(lin)
    out = torch.nn.Linear(64, 1, dtype=torch.float64)
    with torch.no_grad():
        out.weight.copy_(torch.from_numpy(w["w_out"])[None])
        out.bias.fill_(w["b_out"])
    net = torch.nn.Sequential(*layers, out)
    rt = 0.1 * torch.tanh(net(torch.from_numpy(feats))[:, 0])
    assert np.allclose(r, rt.detach().numpy(), rtol=1e-12, atol=1e-15)
    (rt * torch.from_numpy(dl)).sum().backward()
    for l, lin in enumerate(tw):
        assert np.allclose(g["W"][l], lin.weight.grad.numpy(), rtol=1e-10, atol=1e-14)
        assert np.allclose(g["b"][l], lin.bias.grad.numpy(), rtol=1e-10, atol=1e-14)
    assert np.allclose(g["w_out"], out.weight.grad.numpy()[0], rtol=1e-10, atol=1e-14)
    assert g["b_out"] == pytest.approx(float(out.bias.grad), rel=1e-10)

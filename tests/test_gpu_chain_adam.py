"""Fused chain rule + Adam (gm_chain_adam) against the three-call sequence it replaces.

Bar: parameters and both moments bit-identical to clearing a gradient buffer, gm_chain into it
and gm_adam_step on each of the four groups (the gradient is rounded to float as gm_chain
stores it, and both kernels take the same Adam element update).  The chain rule itself is
checked against the FP64 oracle by the backward parity tests, and Adam by the loss/Adam test.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2603_00145_amd import inputs

pytestmark = pytest.mark.gpu
LRS = (1e-3, 1e-3, 5e-3, 5e-2)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    from paper_2603_00145_amd import api as _api
    _api.load()
    return _api


def problem(api, seed, n_g=500, n=33):
    rng = np.random.default_rng(seed)
    g = inputs.init_anisotropic(n, n_g, rng)
    grids = [inputs.stack_grid("axial", n, 9, 1.0, *inputs.random_rigid(rng, 2, 1, n)),
             inputs.stack_grid("coronal", n, 8, 1.0),
             inputs.volume_grid(n)]
    dl = inputs.random_dl_di(grids, rng)
    p = api.GaussParams.from_host(g)
    b = api.Bins(p.n, grids)
    b.bin(p)
    api.grid_partials(p, b, [0, 1, 2], [torch.from_numpy(d).cuda() for d in dl])
    return p, b, rng


def clone(api, p):
    return api.GaussParams(*(t.clone() for t in p.tensors()))


def moments(api, p, rng, zero):
    m, v = api.GaussParams.zeros_like(p), api.GaussParams.zeros_like(p)
    if not zero:
        for a, b in zip(m.tensors(), v.tensors()):
            a.copy_(torch.from_numpy(rng.normal(0, 1e-2, size=tuple(a.shape)).astype(np.float32)))
            b.copy_(torch.from_numpy(rng.uniform(0, 1e-3, size=tuple(b.shape)).astype(np.float32)))
    return m, v


@pytest.mark.parametrize("seed,step,zero", [(0, 1, True), (1, 7, False)])
def test_chain_adam_equals_three_calls(api, seed, step, zero):
    p, b, rng = problem(api, seed)
    m0, v0 = moments(api, p, rng, zero)
    say("chain+adam seed", seed, "step", step)
    # the three-call sequence
    pa, ma, va = clone(api, p), clone(api, m0), clone(api, v0)
    grads = api.GaussParams.zeros_like(p)
    api.chain(pa, b, [0, 1, 2], grads, 0.1, 1.5)
    for prm, gr, mm, vv, lr in zip(pa.tensors(), grads.tensors(), ma.tensors(), va.tensors(), LRS):
        api.adam_step(prm, gr, mm, vv, lr, step)
    # fused
    pb, mb, vb = clone(api, p), clone(api, m0), clone(api, v0)
    api.chain_adam(pb, b, [0, 1, 2], mb, vb, LRS, step, 0.1, 1.5)
    torch.cuda.synchronize()
    for name, x, y in zip(("mean", "quat", "log_scale", "logit"), pa.tensors(), pb.tensors()):
        assert torch.equal(x, y), f"parameter {name} differs"
        assert not torch.equal(x, getattr(p, name)), f"parameter {name} did not move"
    for x, y in zip(ma.tensors() + va.tensors(), mb.tensors() + vb.tensors()):
        assert torch.equal(x, y)


def test_chain_adam_rejects_bad_arguments(api):
    from paper_2603_00145_amd import _lib
    p, b, rng = problem(api, 3, n_g=50, n=17)
    m, v = moments(api, p, rng, True)
    with pytest.raises(_lib.GmError):
        api.chain_adam(p, b, [0, 1, 2], m, v, LRS, 0)                      # step < 1
    with pytest.raises(_lib.GmError):
        api.chain_adam(p, b, [0, 1, 2], m, v, LRS, 1, beta1=1.0)           # beta1 >= 1
    with pytest.raises(_lib.GmError):
        api.chain_adam(p, b, [0, 1, 2], m, v, (1e-3, float("nan"), 1e-3, 1e-3), 1)
    short = api.GaussParams(*(t[:-1] for t in m.tensors()))
    with pytest.raises(_lib.GmError, match="moments"):
        api.chain_adam(p, b, [0, 1, 2], short, v, LRS, 1)


def test_chain_adam_edges(api):
    """No listed grid (only the anisotropy term moves the scales) and no Gaussian at all."""
    p, b, rng = problem(api, 4, n_g=80, n=17)
    m0, v0 = moments(api, p, rng, True)
    pa, ma, va = clone(api, p), clone(api, m0), clone(api, v0)
    grads = api.GaussParams.zeros_like(p)
    api.chain(pa, b, [], grads, 0.5, 1.0)
    for prm, gr, mm, vv, lr in zip(pa.tensors(), grads.tensors(), ma.tensors(), va.tensors(), LRS):
        api.adam_step(prm, gr, mm, vv, lr, 1)
    pb, mb, vb = clone(api, p), clone(api, m0), clone(api, v0)
    api.chain_adam(pb, b, [], mb, vb, LRS, 1, 0.5, 1.0)
    torch.cuda.synchronize()
    for x, y in zip(pa.tensors() + ma.tensors() + va.tensors(),
                    pb.tensors() + mb.tensors() + vb.tensors()):
        assert torch.equal(x, y)
    g0 = inputs.init_anisotropic(17, 1, rng).subset(slice(0, 0))
    p0 = api.GaussParams.from_host(g0)
    b0 = api.Bins(0, [inputs.volume_grid(17)])
    b0.bin(p0)
    m, v = moments(api, p0, rng, True)
    api.chain_adam(p0, b0, [0], m, v, LRS, 1)     # nothing to do, no error
    torch.cuda.synchronize()

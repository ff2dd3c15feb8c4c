"""The training step's entry points on a stream other than the default one.

gm_bin waits for its pair total on an event recorded on the caller's stream (created for that
stream's device), and every other entry point launches on the stream it is given.  One step
(bin, fused render + loss, grid partials, fused chain + Adam) run on a side stream must give
the same bits as on the default stream.
"""
import numpy as np
import pytest
import torch

from paper_2603_00145_amd import inputs

pytestmark = pytest.mark.gpu
LRS = (1e-3, 1e-3, 5e-3, 5e-2)


@pytest.fixture(scope="module")
def api():
    from paper_2603_00145_amd import api as _api
    _api.load()
    return _api


def one_step(api, g, grids, targ):
    p = api.GaussParams.from_host(g)
    m, v = api.GaussParams.zeros_like(p), api.GaussParams.zeros_like(p)
    b = api.Bins(p.n, grids)
    b.bin(p)
    ids = list(range(len(grids)))
    t = [torch.from_numpy(x).cuda() for x in targ]
    loss, dl = api.render_loss(b, ids, t)
    api.grid_partials(p, b, ids, dl)
    api.chain_adam(p, b, ids, m, v, LRS, 1, 0.1, 1.5)
    return b.n_pairs, loss, [x.clone() for x in p.tensors()], [x.clone() for x in dl]


def test_step_on_a_side_stream_equals_default(api):
    rng = np.random.default_rng(11)
    g = inputs.init_anisotropic(29, 400, rng)
    grids = [inputs.stack_grid("axial", 29, 8, 1.0, *inputs.random_rigid(rng, 2, 1, 29)),
             inputs.stack_grid("coronal", 29, 7, 1.0)]
    targ = [rng.normal(0.3, 1.0, size=gr.shape).astype(np.float32) for gr in grids]
    ref = one_step(api, g, grids, targ)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()          # default priority
    with torch.cuda.stream(side):
        got = one_step(api, g, grids, targ)
    side.synchronize()
    assert got[0] == ref[0]
    assert float(got[1]) == float(ref[1])
    for a, r in zip(got[2] + got[3], ref[2] + ref[3]):
        assert torch.equal(a, r)

"""Served requests on the GPU: each result is the same alone and in the mix."""
import numpy as np
import pytest

from paper_2007_12227_amd.inputs import request_trace

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2007_12227_amd import binding
    binding.lib()
    return binding


def test_served_results_equal_alone_results(B):
    from paper_2007_12227_amd.serving import Server, summary
    trace = request_trace(24, seed=11, rate=400.0, n_min=64, n_max=320, steps_min=20, steps_max=150)
    budget = 4 * B.workspace_bytes(trace[0].instance().x, trace[0].instance().p) + (48 << 20)
    srv = Server(budget_bytes=budget, chunk=32, realtime=False, keep_density=True)
    res = srv.run(trace)
    assert len(res) == len(trace)
    assert srv.peak_bytes <= budget or max(r.n for r in res) ** 2 * 12 > budget
    assert srv.batch_rebuilds > 1
    for r in res:
        req = trace[r.rid]
        g = B.grid_for(req.instance())
        g.step(req.instance().dt, req.steps)
        assert np.array_equal(g.density(), r.density), r.rid
        assert r.moments["step"] == req.steps
        g.close()
    s = summary(res)
    print(s)
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_served_grids_share_one_deposit_shape(B):
    """The server gives every grid one deposit launch shape (cut to smaller
    lattices), so a batch's launch does not run small tiles at the LDS of a
    large one; the one-at-a-time baseline keeps each grid's default."""
    from paper_2007_12227_amd.inputs import fel_gaussian, pendulum_band
    from paper_2007_12227_amd.serving import DeviceBackend
    be, plain = DeviceBackend(), DeviceBackend(deposit_tiles=None)
    for inst in (pendulum_band(2048, steps=1), pendulum_band(96, steps=1), fel_gaussian(256, steps=1)):
        g = be.make_grid(inst)
        t = g.tiles()
        assert t["k1"] == (128, 64) and t["threads"] == 512, t  # (planning cuts it to a small lattice)
        g.step(inst.dt, 1)
        g.close()
    g = plain.make_grid(pendulum_band(2048, steps=1))
    assert g.tiles()["k1"] == (128, 128) and g.tiles()["threads"] == 1024
    g.close()

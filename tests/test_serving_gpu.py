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

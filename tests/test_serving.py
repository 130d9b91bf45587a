"""Scheduling logic of the serving loop, on the CPU with a fake device."""
import numpy as np

from paper_2007_12227_amd.inputs import H_FEL, Request, request_trace
from paper_2007_12227_amd.serving import Server, serve_one_at_a_time, summary


class FakeGrid:
    def __init__(self, inst, log):
        self.inst, self.steps, self.closed, self.log = inst, 0, False, log

    def moments(self):
        return {"step": self.steps}

    def density(self):
        return np.full((2, 2), self.steps, dtype=np.float32)

    def close(self):
        self.closed = True


class FakeBatch:
    def __init__(self, grids, log):
        self.grids, self.log = grids, log
        log.append(("batch", len(grids)))

    def step(self, n):
        for g in self.grids:
            assert not g.closed
            g.steps += n

    def close(self):
        pass


class FakeBackend:
    def __init__(self):
        self.log = []

    def footprint(self, inst):
        return inst.x.n * inst.p.n * 12

    def make_grid(self, inst):
        return FakeGrid(inst, self.log)

    def make_batch(self, grids, dts):
        return FakeBatch(grids, self.log)

    def step_alone(self, grid, dt, n):
        grid.steps += n

    def sync(self):
        pass

    def collect(self, grid, keep_density):
        return grid.moments(), grid.density() if keep_density else None, None


def small_trace():
    return request_trace(40, seed=9, rate=1e6, n_min=16, n_max=64, steps_min=5, steps_max=60)


def test_every_request_runs_exactly_its_steps():
    be = FakeBackend()
    res = Server(budget_bytes=10**9, chunk=7, realtime=False, backend=be).run(small_trace())
    assert len(res) == 40
    assert all(r.moments["step"] == r.steps for r in res)
    assert all(r.completed >= r.admitted >= r.arrival for r in res)


def test_budget_is_respected_and_requests_queue():
    be = FakeBackend()
    trace = small_trace()
    budget = 3 * 64 * 64 * 12
    srv = Server(budget_bytes=budget, chunk=16, realtime=False, backend=be)
    res = srv.run(trace)
    assert len(res) == 40 and all(r.moments["step"] == r.steps for r in res)
    assert srv.peak_bytes <= budget
    # several requests shared a batch, and the composition changed over time
    sizes = [n for tag, n in be.log if tag == "batch"]
    assert max(sizes) > 1 and len(set(sizes)) > 1


def test_admission_is_fifo_and_waits_for_arrivals():
    reqs = [Request(0, 0.0, 2, 16, 10, 1), Request(1, 5.0, 2, 16, 10, 2), Request(2, 5.0, H_FEL, 16, 3, 3)]
    be = FakeBackend()
    res = Server(budget_bytes=10**9, chunk=100, realtime=False, backend=be).run(reqs)
    by = {r.rid: r for r in res}
    assert by[1].admitted >= 5.0 and by[2].admitted >= 5.0
    assert by[0].completed < by[1].admitted


def test_one_at_a_time_baseline_and_summary():
    be = FakeBackend()
    res = serve_one_at_a_time(small_trace(), realtime=False, backend=be)
    assert [r.rid for r in res] == sorted(r.rid for r in res)
    s = summary(res)
    assert s["requests"] == 40 and s["node_steps"] > 0 and s["p99_latency_s"] >= s["p50_latency_s"]


def test_request_larger_than_the_budget_is_refused_not_run():
    trace = small_trace()
    be = FakeBackend()
    big = max(trace, key=lambda r: r.n)
    budget = be.footprint(big.instance()) - 1
    res = Server(budget_bytes=budget, chunk=8, realtime=False, backend=be).run(trace)
    assert len(res) == len(trace)
    refused = [r for r in res if r.error]
    assert refused and all(be.footprint(next(q for q in trace if q.rid == r.rid).instance()) > budget
                           for r in refused)
    assert all(r.moments["step"] == r.steps for r in res if not r.error)
    s = summary(res)
    assert s["failed"] == len(refused) and s["requests"] == len(trace) - len(refused)

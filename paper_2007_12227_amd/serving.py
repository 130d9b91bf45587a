"""Continuous-batching request loop over the C interface.

Requests (a Hamiltonian, a lattice, an initial density, a step count) arrive
over time.  Admitted requests stay resident on the device (weights, and for
the FEL the field, live in their grid workspaces) and advance together: each
iteration launches one batched step sequence (``vp_batch_step``) covering
every resident grid.  A request is admitted as soon as it has arrived and its
workspace fits in the HBM budget next to the residents; it joins at the next
iteration boundary.  Finished requests retire at the end of the iteration in
which their step count is reached, freeing their memory.

The device work is done by libvp; this module only schedules it.  ``backend``
is injectable so that the scheduling logic can be tested without a GPU.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Result:
    rid: int
    kind: int
    n: int
    steps: int
    arrival: float
    admitted: float = 0.0
    completed: float = 0.0
    moments: dict = field(default_factory=dict)
    density: np.ndarray | None = None
    error: str | None = None  # why the request failed (its results are then not valid)

    @property
    def latency(self) -> float:
        return self.completed - self.arrival

    @property
    def node_steps(self) -> int:
        return self.n * self.n * self.steps


class DeviceBackend:
    """The libvp device path: grids, batches, synchronisation.

    Every grid gets the same deposit launch shape (`deposit_tiles`: columns,
    rows, threads; the library cuts it to smaller lattices): a batch launches
    one workgroup size and the LDS of its largest tile for every tile, so
    grids of mixed default shapes would run their small tiles at the
    occupancy of the largest.  None keeps each grid's default shape."""

    def __init__(self, deposit_tiles=(128, 64, 512)):
        from . import binding
        self.B = binding
        self.deposit_tiles = deposit_tiles
        binding.lib()

    def footprint(self, inst) -> int:
        return self.B.workspace_bytes(inst.x, inst.p) + 256

    def make_grid(self, inst):
        g = self.B.grid_for(inst)
        if self.deposit_tiles is not None:
            t = self.deposit_tiles
            g.set_tiles((t[0], t[1]), t[2])
        return g

    def make_batch(self, grids, dts):
        return self.B.Batch(grids, dts)

    def collect(self, grid, keep_density: bool):
        """(moments, density or None, error or None) of a finished grid: a
        state the library reports as invalid (non-finite weights, a deposit
        out of its fixed-point range) fails the request."""
        try:
            m = grid.moments()
            d = grid.density() if keep_density else None
            return m, d, None
        except self.B.VpError as e:
            return grid.moments(check_state=False), None, str(e)

    def step_alone(self, grid, dt, n):
        grid.step(dt, n)

    def sync(self):
        import torch
        torch.cuda.current_stream().synchronize()


@dataclass
class _Resident:
    req: object
    inst: object
    grid: object
    remaining: int
    nbytes: int
    result: Result


class Server:
    """Serve a request trace.

    budget_bytes: HBM budget for the resident grid workspaces.
    chunk: most steps advanced per iteration (iterations are also cut at the
      next completion, so no request overshoots its step count).
    realtime: follow the trace's arrival times on the wall clock; otherwise
      time jumps to the next arrival whenever the device would idle.
    keep_density: copy each finished request's weights to the host.
    """

    def __init__(self, budget_bytes: int, chunk: int = 64, realtime: bool = True,
                 keep_density: bool = False, backend=None):
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.realtime = realtime
        self.keep_density = keep_density
        self.backend = backend if backend is not None else DeviceBackend()
        self.iterations = 0
        self.batch_rebuilds = 0
        self.peak_bytes = 0

    def run(self, requests) -> list[Result]:
        be = self.backend
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        resident: list[_Resident] = []
        results: list[Result] = []
        used = 0
        batch = None
        t0 = time.perf_counter()
        offset = 0.0  # virtual time skipped while idle (realtime=False)

        def now() -> float:
            return time.perf_counter() - t0 + offset

        while pending or resident:
            t = now()
            changed = False
            while pending and pending[0].arrival <= t:
                req = pending[0]
                inst = req.instance()
                need = be.footprint(inst)
                if need > self.budget:
                    # can never fit: refused, not run
                    pending.popleft()
                    results.append(Result(req.rid, req.kind, req.n, req.steps, req.arrival, admitted=now(),
                                          completed=now(), error=f"needs {need} bytes, budget {self.budget}"))
                    continue
                if resident and used + need > self.budget:
                    break  # wait for memory to free up (FIFO admission)
                pending.popleft()
                res = Result(req.rid, req.kind, req.n, req.steps, req.arrival, admitted=now())
                resident.append(_Resident(req, inst, be.make_grid(inst), req.steps, need, res))
                used += need
                changed = True
            self.peak_bytes = max(self.peak_bytes, used)
            if not resident:
                if pending:
                    wait = pending[0].arrival - now()
                    if wait > 0:
                        if self.realtime:
                            time.sleep(wait)
                        else:
                            offset += wait
                continue
            if changed or batch is None:
                if batch is not None:
                    batch.close()
                batch = be.make_batch([r.grid for r in resident], [r.inst.dt for r in resident])
                self.batch_rebuilds += 1
            s = min(self.chunk, min(r.remaining for r in resident))
            try:
                batch.step(s)
            except getattr(getattr(be, "B", None), "VpError", ()) as e:
                if getattr(e, "code", None) != -7:
                    raise
                # a resident's deposit left its fixed-point range: fail the
                # residents whose state says so, keep serving the others
                be.sync()
                batch.close()
                batch = None
                keep = []
                for r in resident:
                    m, _, err = be.collect(r.grid, False)
                    if err:
                        r.result.completed, r.result.moments, r.result.error = now(), m, err
                        r.grid.close()
                        used -= r.nbytes
                        results.append(r.result)
                    else:
                        keep.append(r)
                resident = keep
                continue
            self.iterations += 1
            for r in resident:
                r.remaining -= s
            done = [r for r in resident if r.remaining == 0]
            if done:
                be.sync()
                batch.close()
                batch = None
                tdone = now()
                for r in done:
                    r.result.completed = tdone
                    r.result.moments, r.result.density, r.result.error = be.collect(r.grid, self.keep_density)
                    r.grid.close()
                    used -= r.nbytes
                    results.append(r.result)
                resident = [r for r in resident if r.remaining > 0]
        if batch is not None:
            batch.close()
        return results


def serve_one_at_a_time(requests, realtime: bool = True, backend=None) -> list[Result]:
    """The plain baseline: requests run alone, first come first served, each
    grid with its own default deposit shape."""
    be = backend if backend is not None else DeviceBackend(deposit_tiles=None)
    out = []
    t0 = time.perf_counter()
    offset = 0.0
    for req in sorted(requests, key=lambda r: r.arrival):
        t = time.perf_counter() - t0 + offset
        if req.arrival > t:
            if realtime:
                time.sleep(req.arrival - t)
            else:
                offset += req.arrival - t
        inst = req.instance()
        res = Result(req.rid, req.kind, req.n, req.steps, req.arrival,
                     admitted=time.perf_counter() - t0 + offset)
        g = be.make_grid(inst)
        be.step_alone(g, inst.dt, req.steps)
        be.sync()
        res.completed = time.perf_counter() - t0 + offset
        res.moments, _, res.error = be.collect(g, False)
        g.close()
        out.append(res)
    return out


def summary(results: list[Result], wall: float | None = None) -> dict:
    failed = [r for r in results if r.error]
    results = [r for r in results if not r.error]
    lat = np.array([r.latency for r in results])
    work = float(sum(r.node_steps for r in results))
    if wall is None:
        wall = max(r.completed for r in results) - min(r.arrival for r in results)
    return {"requests": len(results), "failed": len(failed), "node_steps": work, "wall_s": wall,
            "node_steps_per_s": work / wall if wall > 0 else float("nan"),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean())}

"""Batched execution: one launch of each per-step kernel covers every tile of
every grid.  The deposit accumulates in integers and the solve has no atomics,
so every instance must come out bit-identical to the same instance run alone;
sampled small instances are also checked against the FP64 oracle."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2007_12227_amd.inputs import FEL_RK4, batch_instances, fel_gaussian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2007_12227_amd import binding
    binding.lib()
    return binding


def alone(B, inst, steps):
    g = B.grid_for(inst)
    g.step(inst.dt, steps)
    out = g.density()
    g.close()
    return out


def test_ragged_mixed_batch_equals_alone(B):
    insts = batch_instances(24, seed=40, steps=30, n_min=48, n_max=300)
    insts += [fel_gaussian(96, 30, npp=128), fel_gaussian(160, 30, npp=64)]
    rk = fel_gaussian(112, 30, npp=96)   # and one advanced by the Runge-Kutta integrator
    insts.append(dataclasses.replace(rk, ham=dataclasses.replace(rk.ham, integrator=FEL_RK4, fel_sigma2=0.3)))
    grids = [B.grid_for(i) for i in insts]
    grids[3].set_tiles((32, 8), 128)       # per-instance tile shapes in one launch,
    grids[5].set_tiles((128, 64), 1024)    # which runs at the largest workgroup size
    batch = B.Batch(grids, [i.dt for i in insts])
    batch.step(13)
    batch.step(17)                            # odd split: the parity bookkeeping
    batch.close()
    for k, (g, inst) in enumerate(zip(grids, insts)):
        got = g.density()
        ref_g = B.grid_for(inst)
        if k == 3:
            ref_g.set_tiles((32, 8), 128)
        ref_g.step(inst.dt, 30)
        assert np.array_equal(got, ref_g.density()), k
        assert g.moments()["step"] == 30
        ref_g.close()
        g.close()


def test_batched_workload_256_instances(B):
    """256 pendulum instances, n log-uniform in [64, 1024], 500 steps."""
    insts = batch_instances(256, seed=4, steps=500)
    grids = [B.grid_for(i) for i in insts]
    batch = B.Batch(grids, [i.dt for i in insts])
    batch.step(500)
    batch.close()
    rng = np.random.default_rng(7)
    for k in rng.choice(len(insts), 12, replace=False):
        assert np.array_equal(grids[k].density(), alone(B, insts[k], 500)), k
    small = sorted(range(len(insts)), key=lambda k: insts[k].nodes)[:3]
    for k in small:
        inst = insts[k]
        ref = oracle.run(inst.x, inst.p, inst.ham, inst.w0.astype(np.float32).astype(np.float64),
                         inst.dt, 500).w
        err = oracle.rel_l1(grids[k].density(), ref)
        print(f"instance {k} ({inst.x.n}^2): rel L1 vs oracle {err:.3e}")
        assert err <= 1e-4
    for g in grids:
        g.close()


def test_grid_in_batch_refuses_own_steps(B):
    inst = batch_instances(1, seed=41, steps=5, n_min=64, n_max=64)[0]
    g = B.grid_for(inst)
    batch = B.Batch([g], [inst.dt])
    with pytest.raises(B.VpError) as e:
        g.step(inst.dt, 1)
    assert e.value.code == B.VP_ESTATE
    batch.close()
    g.step(inst.dt, 1)
    g.close()


def test_batch_of_grids_on_different_streams_is_refused(B):
    """A batch runs on one stream: grids on two streams are refused (their
    work would not be ordered)."""
    import torch
    insts = batch_instances(2, seed=42, steps=5, n_min=64, n_max=64)
    side = torch.cuda.Stream()  # default priority
    g0 = B.grid_for(insts[0])
    g1 = B.grid_for(insts[1], stream=side)
    with pytest.raises(B.VpError) as e:
        B.Batch([g0, g1], [i.dt for i in insts])
    assert e.value.code == B.VP_EINVAL
    side.synchronize()
    g1.close()
    g0.close()


def test_batch_autotune_keeps_states_and_results(B):
    """The batch autotuner times candidate launches on the batch itself (shared
    tile shapes, persistent deposit) and restores every state: stepping after
    tuning equals the grids run alone, bitwise, FEL included; a cached choice
    applies to a batch of the same composition."""
    insts = batch_instances(12, seed=41, steps=20, n_min=48, n_max=260)
    insts += [fel_gaussian(96, 20, npp=128)]
    grids = [B.grid_for(i) for i in insts]
    batch = B.Batch(grids, [i.dt for i in insts])
    batch.step(3)
    us = batch.autotune()
    assert us > 0
    cfg = batch.config()
    assert cfg["deposit_threads"] in (256, 512, 1024) and cfg["deposit_tiles"] > 0
    batch.step(17)
    batch.close()
    for k, (g, inst) in enumerate(zip(grids, insts)):
        assert np.array_equal(g.density(), alone(B, inst, 20)), k
        assert g.moments()["step"] == 20
    # the same composition again: the cached choice, no timing
    grids2 = [B.grid_for(i) for i in insts]
    batch2 = B.Batch(grids2, [i.dt for i in insts])
    batch2.autotune(cached=True)
    assert batch2.config() == cfg
    batch2.step(20)
    batch2.close()
    for g, g2 in zip(grids, grids2):
        assert np.array_equal(g.density(), g2.density())
        g.close()
        g2.close()


def test_batch_timed_steps_equal_batch_steps(B):
    """vp_batch_step_timed advances the batch exactly as vp_batch_step (the
    same launches, direct instead of from graphs, parity kept across calls),
    FEL with both integrators included, and reports positive kernel times."""
    insts = batch_instances(6, seed=42, steps=12, n_min=48, n_max=200)
    insts += [fel_gaussian(96, 12, npp=128)]
    rk = fel_gaussian(80, 12, npp=64)
    insts.append(dataclasses.replace(rk, ham=dataclasses.replace(rk.ham, integrator=FEL_RK4)))
    grids = [B.grid_for(i) for i in insts]
    batch = B.Batch(grids, [i.dt for i in insts])
    batch.step(3)
    dep_us, solve_us = batch.step_timed(5)
    assert dep_us > 0 and solve_us > 0
    batch.step(4)
    with pytest.raises(B.VpError) as e:
        batch.step_timed(0)
    assert e.value.code == B.VP_EINVAL
    batch.close()
    for k, (g, inst) in enumerate(zip(grids, insts)):
        assert np.array_equal(g.density(), alone(B, inst, 12)), k
        assert g.moments()["step"] == 12
        g.close()

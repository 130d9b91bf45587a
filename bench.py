#!/usr/bin/env python3
"""Throughput of the phase-space-conservation Vlasov step on one MI355X.

One bench step = one full time step of the hot path (push, B-spline deposit,
mass-matrix solves) over the 2048^2 pendulum with the uniform band start
(|p| <= 2.5, 1% noise, dt 0.02; its full run is 1000 steps).  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-steps/s (push+deposit) vs plain; % HBM roofline; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
ALG_BYTES_PER_NODE = 8  # a step (and each of its kernels) must read one FP32 array and write one
KERNELS = ("k_deposit", "k_solve")
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2007_12227_amd", "csrc", f)
                  for f in ("vp_kernels.hip", "vp_internal.h", "vp_device.h")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_steps(g, dt, steps, warmup, restore=None):
    """Time exactly `steps` steps replayed as the library runs them.  Before the
    timed region: `warmup` steps, then the same `steps` once more (rounded up to
    an even count, so the timed run starts at the same step parity) to build
    every HIP graph the timed run replays; `restore` (optional) then resets
    the state, and a zero-step call plans the step (tables, the FEL's first
    bunching) outside the timed region."""
    import torch
    g.step(dt, warmup)
    g.step(dt, steps + (steps & 1))
    if restore is not None:
        restore()
    g.step(dt, 0)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    g.step(dt, steps)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def bench_fel(binding, steps, integrator=0):
    """1024^2 FEL (Gaussian in energy, A0 = 1e-3, dz = 0.01), tuned launch;
    integrator 0: exact-kick drift-kick-drift, 1: classical Runge-Kutta."""
    import dataclasses

    from paper_2007_12227_amd.inputs import fel_gaussian
    inst = fel_gaussian(1024, steps)
    inst = dataclasses.replace(inst, ham=dataclasses.replace(inst.ham, integrator=integrator))
    g = binding.grid_for(inst)
    g.autotune(inst.dt)

    def restore():  # the timed run starts from the initial state and field
        g.set_hamiltonian(inst.ham)
        g.set_density(inst.w0)

    sec, _ = timed_steps(g, inst.dt, steps, 0, restore)
    m = g.moments()
    g.close()
    name = "fel_gaussian_1024" + ("_rk4" if integrator else "")
    return {"workload": name, "steps": steps, "value": inst.nodes * steps / sec,
            "ms_per_step": 1e3 * sec / steps, "A_abs": abs(complex(m["A_re"], m["A_im"]))}


def bench_spline(binding, name, n, steps, warmup):
    """The headline workload (pendulum band, n^2) with quadratic or cubic
    B-spline basis functions (name): autotuned deposit tiles, graph replay;
    per-kernel times and the negative mass beside the tent basis's after the
    same steps, and the same comparison on the FEL flat-top start."""
    from paper_2007_12227_amd.inputs import pendulum_band
    spline = {"quadratic": binding.BASIS_QUADRATIC, "cubic": binding.BASIS_CUBIC}[name]
    inst = pendulum_band(n)
    out = {"workload": f"pendulum_band_{n}_{name}", "steps": steps}
    for basis, tag in ((spline, ""), (binding.BASIS_TENT, "tent_")):
        g = binding.Grid(inst.x, inst.p)
        g.set_basis(basis)
        g.set_hamiltonian(inst.ham)
        g.set_density(inst.w0)
        if basis == spline:
            g.autotune(inst.dt)
            sec, _ = timed_steps(g, inst.dt, steps, warmup, restore=lambda: g.set_density(inst.w0))
            out.update(value=inst.nodes * steps / sec, ms_per_step=1e3 * sec / steps, tiles=g.tiles()["k1"])
            m = g.moments()  # after `steps` steps from the start, as the tent grid below
            kus = dict(zip(KERNELS, g.step_timed(inst.dt, min(steps, 200))))
            out["kernels_us"] = kus
            out["kernel_roofline_frac"] = {k: ALG_BYTES_PER_NODE * inst.nodes / (v * 1e-6) / 1e9 / HBM_PEAK_GBS
                                           for k, v in kus.items()}
        else:
            g.autotune(inst.dt, cached=True)
            g.step(inst.dt, steps)
            m = g.moments()
        g.close()
        out[tag + "neg_mass_fraction"] = m["neg_mass"] / m["mass"]
    # the FEL start with a hard energy edge (the case whose negative weights
    # the paper discusses), 500 steps at 1024^2, both bases
    from paper_2007_12227_amd.inputs import fel_flattop
    fl = fel_flattop(1024, 500)
    for basis, tag in ((spline, ""), (binding.BASIS_TENT, "tent_")):
        g = binding.Grid(fl.x, fl.p)
        g.set_basis(basis)
        g.set_hamiltonian(fl.ham)
        g.set_density(fl.w0)
        g.step(fl.dt, fl.steps)
        m = g.moments()
        g.close()
        out[tag + "fel_flattop_neg_mass_fraction"] = m["neg_mass"] / m["mass"]
    return out


def bench_batched(binding, steps, count):
    """256 pendulum instances, n log-uniform in [64, 1024], one launch per kernel
    per step for all of them, against each instance run alone (plain)."""
    import torch

    from paper_2007_12227_amd.inputs import batch_instances
    insts = batch_instances(count, seed=4, steps=steps)
    work = sum(i.nodes for i in insts) * steps
    # each grid keeps the deposit shape chosen by its lattice size: the
    # autotuner times a grid alone, where small grids favour shapes that fill
    # the GPU by themselves, which a batch does not need
    grids = [binding.grid_for(i) for i in insts]
    batch = binding.Batch(grids, [i.dt for i in insts])

    def timed():
        batch.step(steps + (steps & 1))  # builds the graphs the timed run replays
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.step(steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    untuned_sec = timed()
    untuned_cfg = batch.config()
    tune_us = batch.autotune()
    sec = timed()
    cfg = batch.config()
    # per-kernel durations of the batched launches (events on the dispatches)
    kus = dict(zip(KERNELS, batch.step_timed(min(steps, 40))))
    batch.close()
    for g in grids:
        g.close()
    # plain: one solve at a time, default tiles, direct launches
    plain_sec = 0.0
    for i in insts:
        g = binding.grid_for(i)
        g.set_launch(False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.step(i.dt, steps)
        torch.cuda.synchronize()
        plain_sec += time.perf_counter() - t1
        g.close()
    workload = f"batched_{count}_pendulum_64_1024"
    alg = ALG_BYTES_PER_NODE * sum(i.nodes for i in insts)  # per launch of either kernel
    prof_us, traffic = batched_profile(workload, cfg)
    roof = {"bound": "hbm", "kernel": "k_deposit", "achieved": alg / (kus["k_deposit"] * 1e-6) / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg / (kus["k_deposit"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "traffic": traffic, "alg_bytes_per_launch": alg, "kernel_us_events": kus["k_deposit"],
            "kernel_us_rocprof": prof_us,
            "frac_rocprof": None if prof_us is None else alg / (prof_us * 1e-6) / 1e9 / HBM_PEAK_GBS}
    return {"workload": workload, "steps": steps,
            "total_nodes": sum(i.nodes for i in insts), "value": work / sec,
            "ms_per_step": 1e3 * sec / steps, "launch": cfg, "autotune_us_per_step": tune_us,
            "kernels_us": kus, "roofline": roof,
            "kernel_roofline_frac": {k: alg / (v * 1e-6) / 1e9 / HBM_PEAK_GBS for k, v in kus.items()},
            "untuned": {"value": work / untuned_sec, "ms_per_step": 1e3 * untuned_sec / steps, "launch": untuned_cfg},
            "plain_value": work / plain_sec, "speedup_vs_plain": plain_sec / sec}


def bench_phase4d(binding, n, npp, steps, tiles=None):
    """The 2D2V phase space (x, y periodic, p_x, p_y in [-3, 3] open), n^2 x npp^2
    nodes, coupled potential V = -cos x - 0.6 cos y - 0.4 cos(x - y), dt 0.05,
    a noisy near-equilibrium start: steps timed after the same number untimed,
    with the starting deposit tile and then with the autotuned one (or with
    `tiles` alone, no autotuning: for profiling one launch shape)."""
    import numpy as np
    import torch

    from paper_2007_12227_amd.inputs import phase4d_axes, phase4d_thermal
    axes = phase4d_axes(n, npp)
    g = binding.Grid4(axes)
    g.set_hamiltonian(binding.H_PENDULUM, 1.0, 0.6, 0.4)
    w = phase4d_thermal(axes)
    g.set_density(w.astype(np.float32))
    s = torch.cuda.current_stream()

    def timed():
        g.step(0.05, steps)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        g.step(0.05, steps)
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    if tiles is not None:
        g.set_tiles(tiles)
    untuned_tiles = g.tiles()
    untuned_sec = timed()
    tune_us = g.autotune(0.05) if tiles is None else None
    sec = timed() if tiles is None else untuned_sec
    kus = g.step_timed(0.05, min(steps, 10))
    nodes = n * n * npp * npp
    tiles = g.tiles()
    g.close()
    return {"workload": f"phase4d_coupled_{n}x{n}x{npp}x{npp}", "steps": steps, "nodes": nodes,
            "value": nodes * steps / sec, "ms_per_step": 1e3 * sec / steps,
            "tiles": tiles, "autotune_us_per_step": tune_us,
            "kernels_us": {"k_deposit4": kus[0], "k_solve4 (four axes)": kus[1]},
            "untuned": {"tiles": untuned_tiles, "value": nodes * steps / untuned_sec,
                        "ms_per_step": 1e3 * untuned_sec / steps}}


def bench_served(binding, nreq, load, capacity, budget_gib):
    """Poisson arrivals of mixed requests (70% pendulum, 30% FEL, n in
    [128, 2048], 100..2000 steps) served with continuous batching under an HBM
    budget, against the one-at-a-time server on the same trace."""
    from paper_2007_12227_amd import serving
    from paper_2007_12227_amd.inputs import request_trace
    probe = request_trace(nreq, seed=5, rate=1.0)
    mean_work = sum(r.n * r.n * r.steps for r in probe) / nreq
    rate = load * capacity / mean_work
    trace = request_trace(nreq, seed=5, rate=rate)
    srv = serving.Server(budget_bytes=int(budget_gib * (1 << 30)), chunk=64, realtime=True)
    res = srv.run(trace)
    out = serving.summary(res)
    base = serving.summary(serving.serve_one_at_a_time(trace, realtime=True))
    out.update({"workload": f"served_{nreq}_mixed", "load": load, "rate_per_s": rate,
                "budget_gib": budget_gib, "iterations": srv.iterations,
                "batch_rebuilds": srv.batch_rebuilds,
                "plain": {k: base[k] for k in ("node_steps_per_s", "p50_latency_s", "p99_latency_s", "wall_s")}})
    return out


def kernel_source_sha():
    """Hash of the kernel sources (kernels and the instance layout they read)."""
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def deposit_shape(tiles):
    """Deposit launch shape as "COLSxROWSxTHREADS"."""
    return "x".join(str(v) for v in (*tiles["k1"], tiles["threads"]))


def profiled_kernel_us(kernel, workload, shape):
    """Average duration (us) of `kernel` in the committed rocprofv3 kernel-trace
    summary of this workload (the one of this deposit launch shape, if there is
    one), or None unless it was taken of the current kernel sources at this
    deposit launch shape."""
    for name in (f"step_kernels_{workload}_{shape}_kernel_trace.txt", f"step_kernels_{workload}_kernel_trace.txt"):
        path = os.path.join(PROFILES, name)
        if not os.path.exists(path):
            continue
        text = open(path).read()
        if (f"kernel source sha256[:16]: {kernel_source_sha()}" not in text
                or f"shape (columns x rows x threads): {shape}" not in text):
            continue
        for line in text.splitlines():
            if not line.startswith("#") and kernel in line.split("(")[0]:
                return float(line.split()[-4])
    return None


def measured_traffic(kernel, workload, shape):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a copy of
    known size), or None if there is none for the current kernel source (and,
    for the deposit, its launch shape: one summary per measured shape)."""
    name = f"{kernel}_{workload}_{shape}" if kernel == "k_deposit" else f"{kernel}_{workload}"
    path = os.path.join(PROFILES, f"{name}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_sha():
        return None
    if kernel == "k_deposit" and vals.get("deposit_shape") != shape:
        return None
    return float(vals["bytes_per_launch"])


def issue_profile(kernel, workload, shape):
    """The committed rocprofv3 SQ-counter summary of `kernel` on this workload
    and deposit launch shape: VALU- and LDS-active cycles as fractions of the
    busy cycles, and wave-instructions per 64 lattice nodes; None unless it
    was taken of the current kernel sources at this shape."""
    path = os.path.join(PROFILES, f"k_deposit_k_solve_{workload}_{shape}_sq_counters.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if f"kernel source sha256[:16]: {kernel_source_sha()}" not in text:
        return None
    vals, cur = {}, None
    for line in text.splitlines():
        if line.startswith("#"):
            continue
        if not line.startswith(" ") and line.endswith(tuple("0123456789")) and ":" in line:
            cur = line.split(":")[0].strip()
            continue
        if cur == kernel and ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = float(v)
    if not vals:
        return None
    return {"valu_active_over_busy": vals.get("sq_active_inst_valu_over_busy_cu_cycles"),
            "lds_active_over_busy": vals.get("sq_active_inst_lds_over_busy_cu_cycles"),
            "valu_insts_per_64_nodes": vals.get("valu_wave_insts_per_64_nodes"),
            "lds_insts_per_64_nodes": vals.get("lds_wave_insts_per_64_nodes"),
            "source": os.path.basename(path)}


def batched_profile(workload, cfg):
    """(mean deposit duration in us, HBM bytes per deposit launch) of the
    batched launch in configuration `cfg` from the committed rocprofv3
    summaries of this workload, each None unless it was taken of the current
    kernel sources in the same launch configuration (dispatch grid, workgroup)."""
    grid = (cfg["deposit_grid"] or cfg["deposit_tiles"]) * cfg["deposit_threads"]
    key = ("k_deposit<4>", str(grid), str(cfg["deposit_threads"]))
    sha = kernel_source_sha()
    us = traffic = None
    path = os.path.join(PROFILES, f"step_kernels_{workload}_kernel_trace.txt")
    if os.path.exists(path):
        text = open(path).read()
        if f"kernel source sha256[:16]: {sha}" in text:
            for line in text.splitlines():
                f = line.split()
                if len(f) == 5 and tuple(f[:3]) == key:
                    us = float(f[4])
    path = os.path.join(PROFILES, f"k_deposit_k_solve_{workload}_hbm_traffic.txt")
    if os.path.exists(path):
        text = open(path).read()
        if f"kernel_source_sha256_16: {sha}" in text:
            for line in text.splitlines():
                f = line.split()
                if len(f) == 7 and f[0] == "config:" and tuple(f[1:4]) == key:
                    traffic = float(f[5])
    return us, traffic


def cpu_baseline(inst, steps):
    import numpy as np

    import oracle
    w = inst.w0.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    oracle.run(inst.x, inst.p, inst.ham, w, inst.dt, steps)
    dt = time.perf_counter() - t0
    return {"value": inst.nodes * steps / dt, "unit": "node-steps/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{steps} steps of the {inst.x.n}x{inst.p.n} pendulum band from its initial state "
                      f"(FP64 C oracle, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=64)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device copy (scale for HBM counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no FEL / batched / served lines)")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--fel-steps", type=int, default=2000)
    ap.add_argument("--spline-steps", type=int, default=1000,
                    help="steps of the quadratic and cubic basis lines")
    ap.add_argument("--phase4d-n", type=int, default=48, help="2D2V line: nodes along x and y")
    ap.add_argument("--phase4d-np", type=int, default=48, help="2D2V line: nodes along p_x and p_y")
    ap.add_argument("--phase4d-steps", type=int, default=20)
    ap.add_argument("--phase4d-tiles", default=None,
                    help="2D2V line: this deposit tile T0xT1xT2xT3 instead of autotuning (profiling)")
    ap.add_argument("--only", choices=("batched", "phase4d", "fel", "fel_rk4"), default=None,
                    help="run only this line (profiling), printing its JSON object")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--serve-overload", type=float, default=1.2,
                    help="a second served run with arrivals above the batched capacity (0: skip)")
    ap.add_argument("--serve-budget-gib", type=float, default=4.0)
    ap.add_argument("--tiles", default=None,
                    help="deposit launch shape COLSxROWSxTHREADS for the tuned path instead of autotuning "
                         "(uniform dispatches for profiling)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain (untuned, no graph) run")
    ap.add_argument("--map", action="store_true",
                    help="read the cached push map instead of pushing every step (for comparison; off by default)")
    ap.add_argument("--basis", choices=("tent", "quadratic", "cubic"), default="tent",
                    help="basis functions of the timed workload (quadratic, cubic: for profiling their kernels)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2007_12227_amd import binding
    from paper_2007_12227_amd.inputs import pendulum_band

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    binding.lib()
    if args.copy_probe:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    p4_tiles = tuple(int(v) for v in args.phase4d_tiles.split("x")) if args.phase4d_tiles else None
    if args.only:
        if args.only == "batched":
            res = bench_batched(binding, args.batch_steps, args.batch_count)
        elif args.only == "phase4d":
            res = bench_phase4d(binding, args.phase4d_n, args.phase4d_np, args.phase4d_steps, p4_tiles)
        else:
            res = bench_fel(binding, args.fel_steps, integrator=int(args.only == "fel_rk4"))
        print(json.dumps(res), flush=True)
        return
    inst = pendulum_band(args.n)
    N = inst.nodes
    basis = {"tent": binding.BASIS_TENT, "quadratic": binding.BASIS_QUADRATIC, "cubic": binding.BASIS_CUBIC}[args.basis]
    workload = f"pendulum_band_{args.n}" + ("" if args.basis == "tent" else f"_{args.basis}")

    def grid_of(inst):
        g = binding.grid_for(inst)
        g.set_basis(basis)
        if args.map:
            g.set_map_cache(True)
        return g


    # plain path: default tiles, one launch per kernel
    plain = plain_s = None
    if not args.no_plain:
        gp = grid_of(inst)
        gp.set_launch(False)
        plain_s, _ = timed_steps(gp, inst.dt, args.steps, args.warmup)
        gp.close()
        plain = N * args.steps / plain_s
        log(f"plain: {plain:.3e} node-steps/s ({1e6 * plain_s / args.steps:.2f} us/step)")

    # tuned path: autotuned deposit tiles, steps replayed from HIP graphs
    g = grid_of(inst)
    if args.tiles:
        tx, ty, nt = (int(v) for v in args.tiles.lower().split("x"))
        g.set_tiles((tx, ty), nt)
        tune_us = None
    else:
        tune_us = g.autotune(inst.dt)
    tiles = g.tiles()
    log(f"tiles: {tiles} (autotune {tune_us} us/step)")
    sec, wall = timed_steps(g, inst.dt, args.steps, args.warmup)
    value = N * args.steps / sec
    log(f"tuned: {value:.3e} node-steps/s ({1e6 * sec / args.steps:.2f} us/step, wall {wall:.3f} s)")

    # per-kernel durations: HIP events recorded on the grid's stream around
    # each launch, averaged over the steps
    kus = dict(zip(KERNELS, g.step_timed(inst.dt, min(args.steps, 200))))
    m = g.moments()
    g.close()
    log("kernels: " + ", ".join(f"{k} {v:.2f} us" for k, v in kus.items()))
    dom = max(kus, key=kus.get)
    alg_bytes = ALG_BYTES_PER_NODE * N  # per launch of either step kernel
    achieved = alg_bytes / (kus[dom] * 1e-6) / 1e9
    traffic = measured_traffic(dom, workload, deposit_shape(tiles))
    prof_us = profiled_kernel_us(dom, workload, deposit_shape(tiles))

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "node-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "nx": args.n, "np": args.n, "dt": inst.dt,
                   "a": 1.0, "deposit_tiles": tiles["k1"], "deposit_threads": tiles["threads"],
                   "launch": "hip-graph", "push_map_cached": args.map},
        "plain": None if plain is None else {"value": plain, "ms_per_step": 1e3 * plain_s / args.steps,
                                             "speedup": value / plain},
        "kernels_us": kus,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes, "kernel_us_events": kus[dom],
                     "kernel_us_rocprof": prof_us,
                     "frac_rocprof": None if prof_us is None else alg_bytes / (prof_us * 1e-6) / 1e9 / HBM_PEAK_GBS},
        # the dominant kernel is bound by instruction issue, not HBM: its SQ counters
        "issue": issue_profile(dom, workload, deposit_shape(tiles)),
        "kernel_roofline_frac": {k: alg_bytes / (v * 1e-6) / 1e9 / HBM_PEAK_GBS for k, v in kus.items()},
        "step_roofline_frac": alg_bytes / (sec / args.steps) / 1e9 / HBM_PEAK_GBS,
        "final_sum_w": m["sum_w"],
    }
    if not args.no_extras:
        line["fel"] = bench_fel(binding, args.fel_steps)
        log(f"fel: {line['fel']}")
        line["fel_rk4"] = bench_fel(binding, args.fel_steps, integrator=1)
        log(f"fel_rk4: {line['fel_rk4']}")
        for name in ("quadratic", "cubic"):
            line[name] = bench_spline(binding, name, args.n, args.spline_steps, args.warmup)
            log(f"{name}: {line[name]}")
        line["phase4d"] = bench_phase4d(binding, args.phase4d_n, args.phase4d_np, args.phase4d_steps, p4_tiles)
        log(f"phase4d: {line['phase4d']}")
        line["batched"] = bench_batched(binding, args.batch_steps, args.batch_count)
        log(f"batched: {line['batched']}")
        line["served"] = bench_served(binding, args.serve_requests, args.serve_load,
                                      line["batched"]["value"], args.serve_budget_gib)
        log(f"served: {line['served']}")
        if args.serve_overload > 0:
            line["served_overload"] = bench_served(binding, args.serve_requests, args.serve_overload,
                                                   line["batched"]["value"], args.serve_budget_gib)
            log(f"served_overload: {line['served_overload']}")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(inst, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""How far apart equally valid FP32 runs of the FEL workload drift.

Runs the FP64 oracle on the 1024^2 FEL Gaussian (the full-run workload) with
its state rounded to float after every step and, on top of that, one of these
per-step perturbations of the size of the rounding any FP32-state
implementation adds:

  random       w <- fl32(w (1 + eps u)), u uniform in [-1, 1], a fresh draw per
               node and step (seeds 1-4);
  toward_zero  w <- w rounded to float toward zero (a one-sided rounding: the
               systematic bias of a truncating implementation);
  gain+/gain-  w <- fl32(w (1 +/- eps)) (a systematic per-step scale error of
               the size of one rounding).

The relative L1 distance of each run from the exact oracle run (the stored
samples of oracle_fel_gaussian_1024.npz) at the checkpoints shows from which
step on the standard relative-L1 bar stops being a property of the
implementation.  Calls only the oracle and the seeded input generator; writes
fel_sensitivity.txt.

    python tests/golden/fel_sensitivity.py [--jobs 4]   (about 15 minutes on 8 cores)
"""
import argparse
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

EPS = 1e-7
CHECKPOINTS = (1, 500, 1000, 1500, 2000)
RUNS = [("random", 1), ("random", 2), ("random", 3), ("random", 4),
        ("toward_zero", 0), ("gain+", 0), ("gain-", 0)]


def perturb(model, w, rng):
    if model == "random":
        return (w * (1.0 + EPS * rng.uniform(-1, 1, w.shape))).astype(np.float32).astype(np.float64)
    if model == "toward_zero":
        f = w.astype(np.float32)
        up = np.abs(f.astype(np.float64)) > np.abs(w)
        f[up] = np.nextafter(f[up], np.float32(0))
        return f.astype(np.float64)
    if model == "gain+":
        return (w * (1.0 + EPS)).astype(np.float32).astype(np.float64)
    if model == "gain-":
        return (w * (1.0 - EPS)).astype(np.float32).astype(np.float64)
    raise ValueError(model)


def run(spec):
    model, seed = spec
    import oracle
    from paper_2007_12227_amd.inputs import fel_gaussian
    inst = fel_gaussian(1024)
    ref = np.load(os.path.join(HERE, "oracle_fel_gaussian_1024.npz"))
    stride = int(ref["stride"])
    w = inst.w0.astype(np.float32).astype(np.float64)
    l1_w0 = float(np.abs(w[::stride, ::stride]).sum())
    N0 = w.sum()
    A = complex(inst.ham.A_re, inst.ham.A_im)
    rng = np.random.default_rng(seed)
    out = []
    for k in range(1, max(CHECKPOINTS) + 1):
        # the oracle's FP32-state step (rounded to float), then the perturbation
        r = oracle.run(inst.x, inst.p, inst.ham, w, inst.dt, 1, A0=A, N0=N0,
                       round_fp32=model != "toward_zero")
        w, A = perturb(model, r.w, rng), r.A
        if k in CHECKPOINTS:
            exp = ref[f"sample_{k}"].astype(np.float64)
            got = w[::stride, ::stride]
            diff = float(np.abs(got - exp).sum())
            err = diff / float(np.abs(exp).sum())
            dA = abs(A - complex(*ref[f"A_{k}"])) / abs(complex(*ref[f"A_{k}"]))
            out.append((model, seed, k, err, diff / l1_w0, dA))
            print(f"{model} seed {seed} step {k}: rel L1 {err:.3e}  vs ||w0||_1 {diff / l1_w0:.3e}  "
                  f"|dA|/|A| {dA:.2e}", flush=True)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    args = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", str(max(1, 8 // args.jobs)))
    with ProcessPoolExecutor(args.jobs) as ex:
        rows = [r for res in ex.map(run, RUNS) for r in res]
    with open(os.path.join(HERE, "fel_sensitivity.txt"), "w") as f:
        f.write(f"# FEL 1024^2: FP32-state oracle runs with per-step perturbations, eps = {EPS:g}\n")
        f.write("# model seed step rel_l1_vs_exact rel_l1_vs_w0 rel_err_A\n")
        for model, seed, k, err, err0, dA in rows:
            f.write(f"{model} {seed} {k} {err:.6e} {err0:.6e} {dA:.6e}\n")

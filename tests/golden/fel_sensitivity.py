"""How far apart two equally valid FP32 runs of the FEL workload drift.

Runs the FP64 oracle on the 1024^2 FEL Gaussian (the full-run workload) with
its state rounded to float after every step and, on top of that, multiplied
by (1 + eps u), u uniform in [-1, 1], a fresh draw per node and step: the
size of the per-step differences between implementations that all keep an
FP32 state.  Two seeds give two such runs; the relative L1 distance of each
from the exact oracle run (the stored samples of oracle_fel_gaussian_1024.npz)
at the checkpoints shows from which step on the standard relative-L1 bar stops
being a property of the implementation.  Calls only the oracle and the seeded
input generator; writes fel_sensitivity.txt.

    python tests/golden/fel_sensitivity.py      (about 5 minutes on 8 cores)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2007_12227_amd.inputs import fel_gaussian  # noqa: E402

EPS = 1e-7
SEEDS = (1, 2)
CHECKPOINTS = (1, 500, 1000)


def run(seed):
    inst = fel_gaussian(1024)
    ref = np.load(os.path.join(HERE, "oracle_fel_gaussian_1024.npz"))
    stride = int(ref["stride"])
    w = inst.w0.astype(np.float32).astype(np.float64)
    N0 = w.sum()
    A = complex(inst.ham.A_re, inst.ham.A_im)
    rng = np.random.default_rng(seed)
    out = []
    for k in range(1, max(CHECKPOINTS) + 1):
        r = oracle.run(inst.x, inst.p, inst.ham, w, inst.dt, 1, A0=A, N0=N0, round_fp32=True)
        w, A = r.w, r.A
        w = (w * (1.0 + EPS * rng.uniform(-1, 1, w.shape))).astype(np.float32).astype(np.float64)
        if k in CHECKPOINTS:
            exp = ref[f"sample_{k}"].astype(np.float64)
            got = w[::stride, ::stride]
            err = float(np.abs(got - exp).sum() / np.abs(exp).sum())
            dA = abs(A - complex(*ref[f"A_{k}"])) / abs(complex(*ref[f"A_{k}"]))
            out.append((seed, k, err, dA))
            print(f"seed {seed} step {k}: rel L1 {err:.3e}  |dA|/|A| {dA:.2e}", flush=True)
    return out


if __name__ == "__main__":
    rows = [r for s in SEEDS for r in run(s)]
    with open(os.path.join(HERE, "fel_sensitivity.txt"), "w") as f:
        f.write(f"# FEL 1024^2: FP32-state oracle runs with per-step relative noise eps = {EPS:g}\n")
        f.write("# seed step rel_l1_vs_exact rel_err_A\n")
        for seed, k, err, dA in rows:
            f.write(f"{seed} {k} {err:.6e} {dA:.6e}\n")

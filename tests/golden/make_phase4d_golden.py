"""Write the FP64 oracle's one-step result of the 2D2V workload at its
benchmark size (48^4 nodes, coupled potential, dt 0.05) as samples: a strided
sub-lattice, four full lines (one along each axis) through nodes on both sides
of deposit-tile seams, and the full-array sum and L1 norm.  The oracle takes
several minutes at this size, too slow inside a test.  Calls only the oracle and
the seeded input generator.

    python tests/golden/make_phase4d_golden.py      (about 5 minutes)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import phase4d as P4  # noqa: E402
from paper_2007_12227_amd.inputs import phase4d_axes, phase4d_thermal  # noqa: E402

N, NP, DT, STRIDE = 48, 48, 0.05, 4
HAM = P4.Ham4(P4.H4_POTENTIAL, a=1.0, b=0.6, c=0.4)
# line anchors [py, px, y, x]: each lies next to a seam of the default
# 16 x 16 x 8 x 8 deposit tiles on the other three axes
ANCHOR = (23, 24, 16, 15)


def lines(w):
    py, px, y, x = ANCHOR
    return {"line_x": w[py, px, y, :], "line_y": w[py, px, :, x], "line_px": w[py, :, y, x],
            "line_py": w[:, px, y, x]}


if __name__ == "__main__":
    axes = phase4d_axes(N, NP)
    w0 = phase4d_thermal(axes).astype(np.float32).astype(np.float64)  # the FP32 input the GPU receives
    w1 = P4.step(axes, HAM, DT, w0)
    out = {"n": np.array(N), "np": np.array(NP), "dt": np.array(DT), "stride": np.array(STRIDE),
           "ham": np.array([HAM.a, HAM.b, HAM.c]), "anchor": np.array(ANCHOR),
           "sample": w1[::STRIDE, ::STRIDE, ::STRIDE, ::STRIDE].astype(np.float32),
           "sum": np.array(w1.sum()), "l1": np.array(np.abs(w1).sum()), "sum_w0": np.array(w0.sum())}
    out.update({k: v.astype(np.float32) for k, v in lines(w1).items()})
    np.savez_compressed(os.path.join(HERE, "oracle_phase4d_coupled_48.npz"), **out)
    print("sum", out["sum"], "l1", out["l1"], "sample", out["sample"].shape)

"""The stored oracle samples are what the oracle computes (regression pin of
the fixtures, on the case cheap enough to recompute here)."""
import os

import numpy as np

import oracle
from paper_2007_12227_amd.inputs import pendulum_gaussian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_stored_pendulum_gaussian_128_matches_oracle():
    ref = np.load(os.path.join(GOLDEN, "oracle_pendulum_gaussian_128.npz"))
    inst = pendulum_gaussian(128)
    w = inst.w0.astype(np.float32).astype(np.float64)
    done = 0
    for s in ref["steps"]:
        w = oracle.run(inst.x, inst.p, inst.ham, w, inst.dt, int(s) - done).w
        done = int(s)
        np.testing.assert_allclose(w.astype(np.float32), ref[f"sample_{s}"], rtol=0, atol=0)
        assert abs(w.sum() - float(ref[f"sum_{s}"])) < 1e-9 * abs(w.sum())


def test_stored_fixtures_are_consistent():
    for name in ("pendulum_band_2048", "fel_gaussian_1024", "fel_gaussian_1024_rk4"):
        ref = np.load(os.path.join(GOLDEN, f"oracle_{name}.npz"))
        stride = int(ref["stride"])
        for s in ref["steps"]:
            samp = ref[f"sample_{s}"]
            assert samp.dtype == np.float32 and samp.shape == (2048 // stride if "2048" in name else 1024 // stride,) * 2
            # the FP32 floor grows with the step count and stays below the 1e-4 bar
            assert 0 < float(ref[f"fp32_floor_{s}"]) < 1e-4

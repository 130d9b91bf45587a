"""Comparison of a GPU result with the oracle's, shared by the GPU parity tests.

Two bounds, both required: the relative L1 distance (the method's bar) and
the largest node error relative to the largest weight, which a defect
confined to a few tiles (a seam, one solve window) cannot hide in."""
import numpy as np


def step_errors(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.abs(got - ref)
    rel_l1 = float(d.sum() / np.abs(ref).sum())
    rel_max = float(d.max() / np.abs(ref).max())
    return rel_l1, rel_max, np.unravel_index(int(np.argmax(d)), d.shape)


def assert_step_parity(got, ref, tol=1e-5, tol_max=None, label=""):
    """rel L1 <= tol and max|got - ref| <= tol_max max|ref| (tol_max defaults
    to tol); prints both and the worst node."""
    tol_max = tol if tol_max is None else tol_max
    rel_l1, rel_max, at = step_errors(got, ref)
    print(f"{label} rel L1 {rel_l1:.2e}  max/max {rel_max:.2e} at {tuple(int(v) for v in at)}", flush=True)
    assert rel_l1 <= tol, (rel_l1, tol)
    assert rel_max <= tol_max, (rel_max, tol_max, at)

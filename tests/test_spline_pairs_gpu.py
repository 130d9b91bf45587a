"""The spline deposits add the taps of a work unit's two rows (lattice rows
2m, 2m + 1 of one column) as one window when the two sources move by the same
whole cells along p and by at most one apart along x, and source by source
otherwise.  These cases drive each path against the FP64 spline oracle and
check that the result does not depend on the tiling (odd tile heights make
boxes start at odd rows, which the kernel aligns down)."""
import numpy as np
import pytest

import oracle
from _parity import assert_step_parity
from oracle import spline_basis as Q
from paper_2007_12227_amd.inputs import H_FREE, H_PENDULUM, Axis, Hamiltonian, pendulum_axes, rng

pytestmark = pytest.mark.gpu

NODE_TOL = 4.1e-5  # the cubic basis's conditioning bound on a node (the cubic parity tests)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2007_12227_amd import binding
    binding.lib()
    return binding


def run(B, basis, x, p, ham, w, dt, tiles=None):
    g = B.Grid(x, p)
    g.set_basis(basis)
    if tiles:
        g.set_tiles(tiles[:2], tiles[2])
    g.set_hamiltonian(ham)
    g.set_density(w)
    g.step(dt, 1)
    out = g.density().astype(np.float64)
    g.close()
    return out


def reference(x, p, ham, w, dt, degree):
    du, dv = oracle.push(x, p, ham, dt)
    return Q.step(x, p, du, dv, w.astype(np.float64), degree)


def tilings(basis, B):
    threads = 768 if basis == B.BASIS_CUBIC else 1024
    return [None, (32, 7, 256), (64, 5, 512), (24, 9, 64), (96, 33, threads)]


@pytest.mark.parametrize("basis_name", ["quadratic", "cubic"])
@pytest.mark.parametrize("rows_apart", [0.4, 1.0, 2.5])
def test_drift_gradient(B, basis_name, rows_apart):
    """Free streaming where neighbouring rows' drifts differ by rows_apart
    cells: 0.4 (pairs merge, mostly with equal columns), 1.0 (every pair
    merges one column apart), 2.5 (no pair merges)."""
    basis = B.BASIS_QUADRATIC if basis_name == "quadratic" else B.BASIS_CUBIC
    x, p = Axis(0.0, 12.0, 96, True), Axis(-1.5, 1.5, 61, False)
    dt = rows_apart * x.h / p.h
    w = (0.5 + rng(101).random((p.n, x.n))).astype(np.float32)
    ham = Hamiltonian(H_FREE)
    ref = reference(x, p, ham, w, dt, 2 if basis_name == "quadratic" else 3)
    first = None
    for t in tilings(basis, B):
        got = run(B, basis, x, p, ham, w, dt, t)
        assert_step_parity(got, ref, tol_max=NODE_TOL, label=f"{basis_name} {rows_apart} {t}")
        if first is None:
            first = got
        assert np.array_equal(got, first), t


@pytest.mark.parametrize("basis_name", ["quadratic", "cubic"])
def test_strong_kick_mixes_both_paths(B, basis_name):
    """A pendulum kick strong enough that the whole-cell kick of many row
    pairs differs between their rows: merged and source-by-source pairs in
    the same wavefronts."""
    basis = B.BASIS_QUADRATIC if basis_name == "quadratic" else B.BASIS_CUBIC
    x, p = pendulum_axes(120, 90)
    ham = Hamiltonian(H_PENDULUM, a=6.0)
    dt = 0.3
    w = (0.5 + rng(102).random((p.n, x.n))).astype(np.float32)
    du, dv = oracle.push(x, p, ham, dt)
    kv = np.floor(dv)
    share = float(np.mean(kv[0::2][: kv.shape[0] // 2] != kv[1::2][: kv.shape[0] // 2]))
    assert share > 0.05, share  # the case does exercise the source-by-source path
    ref = Q.step(x, p, du, dv, w.astype(np.float64), 2 if basis_name == "quadratic" else 3)
    first = None
    for t in tilings(basis, B):
        got = run(B, basis, x, p, ham, w, dt, t)
        assert_step_parity(got, ref, tol_max=NODE_TOL, label=f"{basis_name} kick {t}")
        if first is None:
            first = got
        assert np.array_equal(got, first), t

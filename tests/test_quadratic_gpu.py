"""Quadratic B-spline basis functions on the GPU (6x6 quintic-tap deposit and
the pentadiagonal solve) against the FP64 quadratic-basis oracle, through the
C interface.  Bars as for tents: relative L1 <= 1e-5 after one step from the
same weights, <= 1e-4 after a run.  Lattices span several 80-node solve tiles
with ragged tails, and lattices narrower than one solve window."""
import numpy as np
import pytest

import oracle
from _parity import assert_step_parity
from oracle import spline_basis as Q
from paper_2007_12227_amd.inputs import (FEL_RK4, H_FEL, H_FREE, H_PENDULUM, H_SHO_EXACT, Axis, Hamiltonian,
                                         fel_gaussian, gaussian, pendulum_axes, pendulum_band, rng)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2007_12227_amd import binding
    binding.lib()
    return binding


def quad_grid(B, x, p, ham, w, tiles=None, graph=True):
    g = B.Grid(x, p)
    g.set_basis(B.BASIS_QUADRATIC)
    if tiles:
        g.set_tiles(tiles[:2], tiles[2] if len(tiles) > 2 else 0)
    g.set_launch(graph)
    g.set_hamiltonian(ham)
    g.set_density(np.ascontiguousarray(w, dtype=np.float32))
    return g


def gpu_steps(B, x, p, ham, w, dt, steps, tiles=None, graph=True):
    g = quad_grid(B, x, p, ham, w, tiles, graph)
    g.step(dt, steps)
    out = g.density().astype(np.float64)
    m = g.moments()
    g.close()
    return out, m


def oracle_step(x, p, ham, w32, dt):
    du, dv = oracle.push(x, p, ham, dt)
    return Q.step(x, p, du, dv, w32.astype(np.float64))


def case(kind):
    if kind == H_SHO_EXACT:
        x, p = Axis(-4, 4, 130, False), Axis(-4, 4, 171, False)
        return x, p, Hamiltonian(kind, omega=1.0), 0.4, gaussian(x, p, 1.0, -0.5, 0.6)
    x, p = pendulum_axes(200, 170)
    w = gaussian(x, p, 0.3, 0.8, 0.5) + 1e-3 * rng(71).random((p.n, x.n))
    return x, p, Hamiltonian(kind, a=1.3), 0.07, w


@pytest.mark.parametrize("kind", [H_FREE, H_PENDULUM, H_SHO_EXACT])
def test_one_step_each_kind(B, kind):
    x, p, ham, dt, w = case(kind)
    w = w.astype(np.float32)
    got, _ = gpu_steps(B, x, p, ham, w, dt, 1)
    ref = oracle_step(x, p, ham, w, dt)
    assert_step_parity(got, ref, label=f"kind {kind}:")


TILINGS = [None, (64, 16), (24, 5, 64), (200, 24, 1024), (128, 128, 1024)]


def test_deposit_tilings_agree_bitwise(B):
    """The fixed-point tile sums do not depend on the deposit tiling."""
    x, p, ham, dt, w = case(H_PENDULUM)
    w = w.astype(np.float32)
    ref = oracle_step(x, p, ham, w, dt)
    first = None
    for t in TILINGS:
        got, _ = gpu_steps(B, x, p, ham, w, dt, 1, t)
        assert_step_parity(got, ref, label=str(t))
        if first is None:
            first = got
        assert np.array_equal(got, first), t


@pytest.mark.parametrize("nx,np_,periodic", [(4, 64, True), (64, 4, True), (40, 24, False), (7, 130, False),
                                             (90, 300, True), (300, 90, False), (128, 128, False)])
def test_one_step_window_shapes(B, nx, np_, periodic):
    """Lattices narrower than a window (taken whole, both edges exact), windows
    cut inside the lattice, and a periodic axis narrower than the halo."""
    if periodic:
        x, p = pendulum_axes(nx, np_)
        ham, dt = Hamiltonian(H_PENDULUM, a=0.8), 0.05
    else:
        x, p = Axis(-3, 3, nx, False), Axis(-3, 3, np_, False)
        ham, dt = Hamiltonian(H_SHO_EXACT, omega=1.0), 0.3
    w = (0.5 + rng(72).random((np_, nx))).astype(np.float32)
    got, _ = gpu_steps(B, x, p, ham, w, dt, 1)
    assert_step_parity(got, oracle_step(x, p, ham, w, dt))


def test_whole_cell_free_streaming_is_a_row_rotation(B):
    """Row j streams by p_j dt / h_x = j - 8 whole cells: the moved density is in
    the span of the basis, and the step returns it exactly (to FP32 rounding
    of the solve)."""
    x, p = Axis(0.0, 64.0, 64, True), Axis(-8.0, 8.0, 17, False)
    w = (0.5 + rng(73).random((p.n, x.n))).astype(np.float32)
    got, _ = gpu_steps(B, x, p, Hamiltonian(H_FREE), w, 1.0, 1)
    for j in range(p.n):
        assert np.abs(got[j] - np.roll(w[j], j - 8)).max() <= 2e-6, j


def test_no_motion_is_identity_including_open_edges(B):
    x, p = Axis(-4, 4, 100, False), Axis(-4, 4, 130, False)
    w = (0.5 + rng(74).random((130, 100))).astype(np.float32)
    got, _ = gpu_steps(B, x, p, Hamiltonian(H_SHO_EXACT, omega=1.0), w, 0.0, 1)
    assert oracle.rel_l1(got, w.astype(np.float64)) <= 1e-6


@pytest.mark.parametrize("kind", [H_PENDULUM, H_SHO_EXACT])
def test_moments_match_oracle(B, kind):
    x, p, ham, dt, w = case(kind)
    g = quad_grid(B, x, p, ham, w)
    g.step(dt, 3)
    state = g.density().astype(np.float64)
    m = g.moments()
    g.close()
    ref = Q.moments(x, p, ham, state)
    for k in ("sum_w", "mass", "neg_mass", "l1", "entropy", "mean_p", "energy"):
        assert abs(m[k] - ref[k]) <= 1e-9 * max(1.0, abs(ref[k])), (k, m[k], ref[k])
    assert m["step"] == 3


def test_run_pendulum_gaussian_256(B):
    """100 steps of the pendulum (a Gaussian crossing the separatrix), graph
    replay, against the oracle's run."""
    x, p = pendulum_axes(256)
    w0 = gaussian(x, p, 0.0, 1.0, 0.3) + 1e-3 * rng(75).random((256, 256))
    ham = Hamiltonian(H_PENDULUM, a=1.0)
    got, m = gpu_steps(B, x, p, ham, w0, 0.05, 100)
    ref = Q.run(x, p, ham, w0.astype(np.float32).astype(np.float64), 0.05, 100)
    err = oracle.rel_l1(got, ref)
    print(f"pendulum 256^2, 100 steps: rel L1 {err:.3e}; negative mass {m['neg_mass']:.3e} of {m['mass']:.6f}",
          flush=True)
    assert err <= 1e-4


def test_one_step_at_2048_in_the_benchmark_launch(B):
    """The 2048^2 pendulum band, autotuned deposit tiles, as the benchmark
    times it: one step against the oracle."""
    inst = pendulum_band(2048)
    g = quad_grid(B, inst.x, inst.p, inst.ham, inst.w0)
    g.autotune(inst.dt)
    w32 = inst.w0.astype(np.float32)
    g.step(inst.dt, 1)
    got = g.density().astype(np.float64)
    g.close()
    assert_step_parity(got, oracle_step(inst.x, inst.p, inst.ham, w32, inst.dt), label="2048^2 band:")


@pytest.mark.parametrize("integrator", [0, FEL_RK4])
@pytest.mark.parametrize("delta,sigma2", [(0.0, 0.0), (0.3, 0.4)])
def test_fel_one_step(B, delta, sigma2, integrator):
    """One FEL step (exact kick, or Runge-Kutta) with the quadratic basis: the
    state and the new field against the oracle."""
    inst = fel_gaussian(96, 1, npp=160)
    ham = Hamiltonian(H_FEL, A_re=0.02, A_im=-0.01, fel_delta=delta, fel_sigma2=sigma2, integrator=integrator)
    w32 = inst.w0.astype(np.float32)
    g = quad_grid(B, inst.x, inst.p, ham, w32)
    g.step(inst.dt, 1)
    got = g.density().astype(np.float64)
    m = g.moments()
    g.close()
    ref, A = Q.run_fel(inst.x, inst.p, ham, w32.astype(np.float64), inst.dt, 1)
    assert_step_parity(got, ref)
    assert abs(complex(m["A_re"], m["A_im"]) - A) <= 1e-12


@pytest.mark.parametrize("integrator", [0, FEL_RK4])
def test_fel_run_256(B, integrator):
    """200 FEL steps at 256^2 with detuning and space charge (the field grows
    several-fold): state, field and the invariant |A|^2 + <eta> against the
    oracle's run (the bunchings come from the quadratic solve's per-tile
    partials and, for Runge-Kutta, the stage kernel on the quadratic tiles)."""
    inst = fel_gaussian(256, 200)
    ham = Hamiltonian(H_FEL, A_re=1e-3, fel_delta=0.2, fel_sigma2=0.3, integrator=integrator)
    w32 = inst.w0.astype(np.float32)
    g = quad_grid(B, inst.x, inst.p, ham, w32)
    g.step(inst.dt, 200)
    got = g.density().astype(np.float64)
    m = g.moments()
    g.close()
    ref, A = Q.run_fel(inst.x, inst.p, ham, w32.astype(np.float64), inst.dt, 200)
    err = oracle.rel_l1(got, ref)
    Ag = complex(m["A_re"], m["A_im"])
    print(f"FEL 256^2 quadratic (integrator {integrator}), 200 steps: rel L1 {err:.3e}, |A| {abs(Ag):.6e} (oracle {abs(A):.6e})", flush=True)
    assert err <= 1e-4
    assert abs(Ag - A) <= 1e-4 * abs(A)
    eta = inst.p.nodes()[:, None]
    inv_ref = abs(A) ** 2 + float((ref * eta).sum()) / float(w32.astype(np.float64).sum())
    assert abs(m["fel_invariant"] - inv_ref) <= 1e-7


def test_unknown_basis_is_refused(B):
    x, p = pendulum_axes(64)
    g = B.Grid(x, p)
    with pytest.raises(B.VpError) as e:
        g.set_basis(7)
    assert e.value.code == B.VP_EINVAL
    g.close()


def test_batch_of_quadratic_grids_matches_single_runs(B):
    cases = []
    for k, (nx, npp, a) in enumerate([(96, 80, 0.7), (200, 170, 1.3), (64, 130, 1.0)]):
        x, p = pendulum_axes(nx, npp)
        w = (gaussian(x, p, 0.2, 0.3, 0.5) + 1e-3 * rng(76 + k).random((npp, nx))).astype(np.float32)
        cases.append((x, p, Hamiltonian(H_PENDULUM, a=a), w, 0.05))
    singles = [gpu_steps(B, x, p, h, w, dt, 20)[0] for x, p, h, w, dt in cases]
    grids = [quad_grid(B, x, p, h, w) for x, p, h, w, _ in cases]
    bt = B.Batch(grids, [c[4] for c in cases])
    bt.step(20)
    bt.close()
    for g, ref in zip(grids, singles):
        assert np.array_equal(g.density().astype(np.float64), ref)
        g.close()


def test_batch_mixing_bases_is_refused(B):
    x, p = pendulum_axes(64)
    w = (0.5 + rng(79).random((64, 64))).astype(np.float32)
    a = quad_grid(B, x, p, Hamiltonian(H_PENDULUM, a=1.0), w)
    b = B.Grid(x, p)
    b.set_hamiltonian(Hamiltonian(H_PENDULUM, a=1.0))
    b.set_density(w)
    with pytest.raises(B.VpError) as e:
        B.Batch([a, b], [0.05, 0.05])
    assert e.value.code == B.VP_EUNSUPPORTED
    a.close()
    b.close()

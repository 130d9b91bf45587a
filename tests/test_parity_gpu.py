"""GPU (HIP, FP32) vs the FP64 oracle on the same seeded inputs, through the C interface.

Bars: relative L1 <= 1e-5 after one step from the same weights, <= 1e-4 after
a full run (the precision the method is asked to hold in FP32).  Inputs span
several tiles with ragged tails; tile shapes are varied to cover every edge
of the tiling.
"""
import math
import os

import numpy as np
import pytest

import oracle
from _parity import assert_step_parity
import dataclasses

from paper_2007_12227_amd.inputs import (FEL_RK4, H_FEL, H_FREE, H_PENDULUM, H_SHO_EXACT, Axis, Hamiltonian,
                                         fel_flattop, fel_gaussian, gaussian, pendulum_axes, pendulum_band,
                                         pendulum_gaussian, rng)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2007_12227_amd import binding
    binding.lib()
    return binding


def gpu_run(B, x, p, ham, w0, dt, steps, tiles=None, graph=True):
    g = B.Grid(x, p)
    if tiles:
        g.set_tiles(tiles[:2], tiles[2] if len(tiles) > 2 else 0)
    g.set_launch(graph)
    g.set_hamiltonian(ham)
    g.set_density(w0)
    g.step(dt, steps)
    out = g.density().astype(np.float64)
    m = g.moments()
    g.close()
    return out, m


def one_step_ref(x, p, ham, w32, dt):
    return oracle.run(x, p, ham, w32.astype(np.float64), dt, 1).w


# deposit launch shapes (columns, rows[, threads]); the solves use fixed 32-node segments
TILINGS = [None, (64, 16), (24, 5, 64), (200, 24, 1024), (128, 128, 1024)]


@pytest.mark.parametrize("tiles", TILINGS)
def test_one_step_pendulum_ragged(B, tiles):
    x, p = pendulum_axes(200, 150)
    w = (gaussian(x, p, 0.3, 0.8, 0.5) + 1e-3 * rng(31).random((150, 200))).astype(np.float32)
    ham = Hamiltonian(H_PENDULUM, a=1.3)
    got, _ = gpu_run(B, x, p, ham, w, 0.07, 1, tiles)
    ref = one_step_ref(x, p, ham, w, 0.07)
    assert_step_parity(got, ref)


@pytest.mark.parametrize("kind", [H_FREE, H_PENDULUM, H_SHO_EXACT, H_FEL])
def test_one_step_each_kind(B, kind):
    if kind == H_SHO_EXACT:
        x, p = Axis(-4, 4, 130, False), Axis(-4, 4, 97, False)
        ham = Hamiltonian(kind, omega=1.0)
        dt = 0.4
        w = gaussian(x, p, 1.0, -0.5, 0.6)
    elif kind == H_FEL:
        inst = fel_gaussian(96, 1, npp=160)
        x, p, dt, w = inst.x, inst.p, inst.dt, inst.w0
        ham = Hamiltonian(kind, A_re=0.02, A_im=-0.01)
    else:
        x, p = pendulum_axes(144, 100)
        ham = Hamiltonian(kind, a=0.9)
        dt = 0.13
        w = gaussian(x, p, -1.0, 0.5, 0.5) + 1e-3 * rng(32).random((p.n, x.n))
    w = w.astype(np.float32)
    got, _ = gpu_run(B, x, p, ham, w, dt, 1, (64, 16))
    if kind == H_FEL:
        A0 = complex(ham.A_re, ham.A_im)
        ref = oracle.run(x, p, ham, w.astype(np.float64), dt, 1, A0=A0).w
    else:
        ref = one_step_ref(x, p, ham, w, dt)
    assert_step_parity(got, ref)


def test_full_run_pendulum_gaussian_128(B):
    inst = pendulum_gaussian(128)
    w32 = inst.w0.astype(np.float32)
    got, m = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, inst.steps)
    ref = oracle.run(inst.x, inst.p, inst.ham, w32.astype(np.float64), inst.dt, inst.steps).w
    err = oracle.rel_l1(got, ref)
    print(f"pendulum_gaussian_128 200 steps: rel L1 {err:.3e}")
    assert err <= 1e-4
    assert m["step"] == inst.steps


@pytest.mark.parametrize("nx,np_", [(12, 40), (33, 7), (4, 64)])
def test_one_step_small_lattices(B, nx, np_):
    # lattices shorter than one solve segment or its halo: the periodic x line
    # wraps several times, the open p line is cut at both true edges
    x, p = pendulum_axes(nx, np_)
    w = (0.5 + rng(35).random((np_, nx))).astype(np.float32)
    ham = Hamiltonian(H_PENDULUM, a=0.8)
    got, _ = gpu_run(B, x, p, ham, w, 0.05, 1, (16, 8))
    ref = one_step_ref(x, p, ham, w, 0.05)
    assert_step_parity(got, ref)


@pytest.mark.parametrize("nx,np_", [(80, 96), (70, 80), (100, 97), (64, 200), (96, 160)])
def test_one_step_solve_window_paths(B, nx, np_):
    """Lattices whose momentum lines take each of the solve's window cases: a
    whole line shorter than a window (70x80), a line of exactly one window
    whose second tile keeps rows 64..95 (80x96), a window shifted to end at the
    top edge (100x97), interior windows (64x200, 96x160)."""
    x, p = pendulum_axes(nx, np_)
    w = (gaussian(x, p, 0.4, -0.3, 0.7) + 1e-3 * rng(36).random((np_, nx))).astype(np.float32)
    ham = Hamiltonian(H_PENDULUM, a=1.1)
    got, _ = gpu_run(B, x, p, ham, w, 0.06, 1, (32, 16))
    ref = one_step_ref(x, p, ham, w, 0.06)
    assert_step_parity(got, ref)


@pytest.mark.parametrize("nx,np_", [(40, 96), (64, 80), (100, 130), (130, 64)])
def test_one_step_open_x_window_paths(B, nx, np_):
    """The exact rotation needs an open x axis: x lines shorter than a window,
    exactly one window, and windows shifted to end at either edge."""
    x, p = Axis(-4, 4, nx, False), Axis(-4, 4, np_, False)
    ham = Hamiltonian(H_SHO_EXACT, omega=1.0)
    w = (gaussian(x, p, 0.8, -0.4, 0.7) + 1e-3 * rng(37).random((np_, nx))).astype(np.float32)
    got, _ = gpu_run(B, x, p, ham, w, 0.3, 1, (32, 16))
    ref = one_step_ref(x, p, ham, w, 0.3)
    assert_step_parity(got, ref)


def test_graph_and_plain_launches_agree(B):
    inst = pendulum_gaussian(128)
    w32 = inst.w0.astype(np.float32)
    a, _ = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 40, graph=True)
    b, _ = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 40, graph=False)
    assert oracle.rel_l1(a, b) <= 1e-6


def rk4(inst, **kw):
    """The same instance advanced by the Runge-Kutta FEL integrator."""
    return dataclasses.replace(inst, ham=dataclasses.replace(inst.ham, integrator=FEL_RK4, **kw))


@pytest.mark.parametrize("kind", ["pendulum", "fel", "fel_rk4"])
def test_results_bitwise_independent_of_deposit_tiling(B, kind):
    """The deposit sums taps as exact integers, so any tiling and workgroup
    size (each node is pushed by every tile whose source box holds it) gives
    the same bits."""
    inst = pendulum_band(256, steps=30) if kind == "pendulum" else fel_gaussian(192, 30, npp=160)
    if kind == "fel_rk4":
        inst = rk4(inst, fel_sigma2=0.3)
    ref = None
    for k1 in [(64, 32, 256), (128, 16, 512), (24, 5, 64), (200, 24, 1024), (16, 8, 128), (128, 128, 1024),
               (96, 40, 320)]:
        g = B.grid_for(inst)
        g.set_tiles(k1[:2], k1[2])
        g.step(inst.dt, 30)
        got = g.density()
        g.close()
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got, ref), k1


def test_fel_graph_and_plain_launches_agree(B):
    inst = fel_gaussian(192, 40, npp=160)
    w32 = inst.w0.astype(np.float32)
    a, ma = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 40, graph=True)
    b, mb = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 40, graph=False)
    assert np.array_equal(a, b)
    assert (ma["A_re"], ma["A_im"]) == (mb["A_re"], mb["A_im"])


# ---- pins re-run on the GPU path ----

def test_gpu_rotation_quarter_turn_is_permutation(B):
    n, h = 48, 0.25
    half = 0.5 * (n - 1) * h
    x = p = Axis(-half, half, n, False)
    w = rng(33).uniform(-1, 1, (n, n)).astype(np.float32)
    got, _ = gpu_run(B, x, p, Hamiltonian(H_SHO_EXACT, omega=1.0), w, math.pi / 2, 1, (16, 8))
    np.testing.assert_allclose(got, np.rot90(w.astype(np.float64)), atol=2e-6)


def test_gpu_free_streaming_integer_shift(B):
    n, K = 64, 21
    x = Axis(0.0, float(n), n, True)
    p = Axis(-float(K), float(n - 1 - K), n, False)
    w = rng(34).uniform(-1, 1, (n, n)).astype(np.float32)
    got, _ = gpu_run(B, x, p, Hamiltonian(H_FREE), w, 1.0, 3, (16, 8))
    ref = np.stack([np.roll(w[j].astype(np.float64), 3 * (j - K)) for j in range(n)])
    np.testing.assert_allclose(got, ref, atol=2e-6)


def test_gpu_mass_conserved(B):
    x, p = pendulum_axes(256)
    w = gaussian(x, p, 0.5, 0.0, 0.3).astype(np.float32)
    s0 = float(w.astype(np.float64).sum())
    got, m = gpu_run(B, x, p, Hamiltonian(H_PENDULUM, a=1.0), w, 0.05, 400)
    # the taps sum to exactly one and the solve keeps the line mass to ~1e-10:
    # what is left is unbiased rounding
    print(f"mass drift over 400 steps: {(m['sum_w'] - s0) / s0:+.3e}")
    assert abs(m["sum_w"] - s0) <= 2e-7 * s0
    assert abs(got.sum() - s0) <= 2e-7 * s0


def test_moments_match_oracle(B):
    inst = pendulum_gaussian(128)
    w32 = inst.w0.astype(np.float32)
    got, m = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 10)
    ref = oracle.moments(inst.x, inst.p, inst.ham, got)
    for k in ("sum_w", "mass", "neg_mass", "l1", "entropy", "mean_p", "energy"):
        assert m[k] == pytest.approx(ref[k], rel=1e-10, abs=1e-12), k


# ---- FEL ----

def test_fel_run_and_invariant(B):
    inst = fel_gaussian(256, 300, npp=256)
    w32 = inst.w0.astype(np.float32)
    got, m = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 300)
    r = oracle.run(inst.x, inst.p, inst.ham, w32.astype(np.float64), inst.dt, 300)
    err = oracle.rel_l1(got, r.w)
    print(f"fel 256^2 300 steps: rel L1 {err:.3e}, A gpu {m['A_re']:+.6e}{m['A_im']:+.6e}j "
          f"oracle {r.A:.6e}")
    assert err <= 1e-4
    assert abs(complex(m["A_re"], m["A_im"]) - r.A) <= 1e-4 * abs(r.A)
    E0 = 1e-6 + float((w32.astype(np.float64) * inst.p.nodes()[:, None]).sum() / w32.sum())
    assert abs(m["fel_invariant"] - E0) <= 1e-7


def test_fel_detuning_and_space_charge(B):
    """The full FEL model of eqs. 13a-c: detuning in the phase drift, space
    charge in the kick; against the oracle, with the invariant |A|^2 + <eta>."""
    base = fel_gaussian(256, 200, npp=256)
    ham = Hamiltonian(H_FEL, A_re=1e-3, fel_delta=0.3, fel_sigma2=0.4)
    w32 = base.w0.astype(np.float32)
    got, m = gpu_run(B, base.x, base.p, ham, w32, base.dt, 200)
    r = oracle.run(base.x, base.p, ham, w32.astype(np.float64), base.dt, 200)
    err = oracle.rel_l1(got, r.w)
    print(f"fel delta 0.3 sigma2 0.4, 200 steps: rel L1 {err:.3e}, A gpu {m['A_re']:+.6e}{m['A_im']:+.6e}j "
          f"oracle {r.A:.6e}")
    assert err <= 1e-4
    assert abs(complex(m["A_re"], m["A_im"]) - r.A) <= 1e-4 * abs(r.A)
    E0 = 1e-6 + float((w32.astype(np.float64) * base.p.nodes()[:, None]).sum() / w32.sum())
    assert abs(m["fel_invariant"] - E0) <= 1e-7


def test_fel_flattop_start(B):
    """The hard-edged start (|eta| <= 0.1): the projection rings at the edges
    and makes negative weights; the GPU follows the oracle, negative mass
    included."""
    inst = fel_flattop(256, 200)
    w32 = inst.w0.astype(np.float32)
    got, m = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 200)
    r = oracle.run(inst.x, inst.p, inst.ham, w32.astype(np.float64), inst.dt, 200)
    err = oracle.rel_l1(got, r.w)
    ref = oracle.moments(inst.x, inst.p, inst.ham, r.w, r.A, N0=float(w32.astype(np.float64).sum()))
    print(f"fel flat-top 200 steps: rel L1 {err:.3e}, neg mass gpu {m['neg_mass']:.6e} oracle {ref['neg_mass']:.6e}")
    assert err <= 1e-4
    assert ref["neg_mass"] > 0.0
    assert abs(m["neg_mass"] - ref["neg_mass"]) <= 1e-4 * ref["l1"]


# ---- FEL by the Runge-Kutta integrator ----

def test_fel_rk4_one_step(B):
    """One Runge-Kutta step (four stage bunchings) of the full model from the
    same FP32 weights: the state to the one-step bar and the field to FP64
    rounding (both sides form every bunching in FP64 from the same weights)."""
    inst = fel_gaussian(96, 1, npp=160)
    ham = Hamiltonian(H_FEL, A_re=0.02, A_im=-0.01, fel_delta=0.3, fel_sigma2=0.4, integrator=FEL_RK4)
    w32 = inst.w0.astype(np.float32)
    got, m = gpu_run(B, inst.x, inst.p, ham, w32, inst.dt, 1, (64, 16))
    r = oracle.run(inst.x, inst.p, ham, w32.astype(np.float64), inst.dt, 1)
    assert_step_parity(got, r.w)
    assert abs(complex(m["A_re"], m["A_im"]) - r.A) <= 1e-12


@pytest.mark.parametrize("delta,sigma2", [(0.0, 0.0), (0.3, 0.4)])
def test_fel_rk4_run(B, delta, sigma2):
    """200 Runge-Kutta steps through the start of the exponential growth,
    against the oracle: state, field and the invariant |A|^2 + <eta> (which
    the method keeps to its order, not exactly)."""
    base = fel_gaussian(256, 200, npp=256)
    ham = Hamiltonian(H_FEL, A_re=1e-3, fel_delta=delta, fel_sigma2=sigma2, integrator=FEL_RK4)
    w32 = base.w0.astype(np.float32)
    got, m = gpu_run(B, base.x, base.p, ham, w32, base.dt, 200)
    r = oracle.run(base.x, base.p, ham, w32.astype(np.float64), base.dt, 200)
    ref = oracle.moments(base.x, base.p, ham, r.w, r.A, N0=float(w32.astype(np.float64).sum()))
    err = oracle.rel_l1(got, r.w)
    print(f"fel rk4 delta {delta} sigma2 {sigma2}, 200 steps: rel L1 {err:.3e}, "
          f"A gpu {m['A_re']:+.6e}{m['A_im']:+.6e}j oracle {r.A:.6e}")
    assert err <= 1e-4
    assert abs(complex(m["A_re"], m["A_im"]) - r.A) <= 1e-4 * abs(r.A)
    assert abs(m["fel_invariant"] - ref["fel_invariant"]) <= 1e-7


def test_fel_rk4_graph_and_plain_launches_agree(B):
    inst = rk4(fel_gaussian(192, 40, npp=160))
    w32 = inst.w0.astype(np.float32)
    a, ma = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 40, graph=True)
    b, mb = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 40, graph=False)
    assert np.array_equal(a, b)
    assert (ma["A_re"], ma["A_im"]) == (mb["A_re"], mb["A_im"])


def test_fel_rk4_step_size_change(B):
    """A new dz re-plans the tables and recomputes the state's bunchings: 20
    steps at dz then 20 at dz/2 match the oracle run the same way."""
    inst = rk4(fel_gaussian(128, 40, npp=160), fel_sigma2=0.2)
    w32 = inst.w0.astype(np.float32)
    g = B.grid_for(dataclasses.replace(inst, w0=w32))
    g.step(inst.dt, 20)
    g.step(0.5 * inst.dt, 20)
    got, m = g.density().astype(np.float64), g.moments()
    g.close()
    N0 = float(w32.astype(np.float64).sum())
    r1 = oracle.run(inst.x, inst.p, inst.ham, w32.astype(np.float64), inst.dt, 20)
    r2 = oracle.run(inst.x, inst.p, inst.ham, r1.w, 0.5 * inst.dt, 20, A0=r1.A, N0=N0)
    assert oracle.rel_l1(got, r2.w) <= 1e-4
    assert abs(complex(m["A_re"], m["A_im"]) - r2.A) <= 1e-4 * abs(r2.A)


# ---- full sizes ----

def test_one_step_full_size_pendulum_band_2048(B):
    inst = pendulum_band(2048)
    w32 = inst.w0.astype(np.float32)
    got, _ = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 1)
    ref = one_step_ref(inst.x, inst.p, inst.ham, w32, inst.dt)
    assert_step_parity(got, ref)


def test_one_step_full_size_fel_rk4_1024(B):
    inst = rk4(fel_gaussian(1024), fel_sigma2=0.2)
    w32 = inst.w0.astype(np.float32)
    got, m = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 1)
    r = oracle.run(inst.x, inst.p, inst.ham, w32.astype(np.float64), inst.dt, 1)
    assert_step_parity(got, r.w)
    assert abs(complex(m["A_re"], m["A_im"]) - r.A) <= 1e-12


def test_one_step_full_size_fel_1024(B):
    inst = fel_gaussian(1024)
    w32 = inst.w0.astype(np.float32)
    got, _ = gpu_run(B, inst.x, inst.p, inst.ham, w32, inst.dt, 1)
    ref = oracle.run(inst.x, inst.p, inst.ham, w32.astype(np.float64), inst.dt, 1).w
    assert_step_parity(got, ref)


@pytest.mark.parametrize("basis", [0, 1, 2])
@pytest.mark.parametrize("kind", [H_FREE, H_PENDULUM, H_SHO_EXACT])
def test_cached_push_map_is_bitwise_the_push(B, kind, basis):
    """A static Hamiltonian's push cached once per plan (the time-invariant map)
    gives bitwise the results of pushing every step, for every basis."""
    if kind == H_SHO_EXACT:
        x, p = Axis(-3.0, 3.0, 150, False), Axis(-3.0, 3.0, 130, False)
        ham, dt = Hamiltonian(H_SHO_EXACT, omega=1.0), 0.2
    else:
        x, p = pendulum_axes(150, 130)
        ham, dt = Hamiltonian(kind, a=1.1), 0.07
    w = (gaussian(x, p, 0.3, 0.5, 0.6) + 1e-3 * rng(71).random((p.n, x.n))).astype(np.float32)
    out = []
    for cached in (True, False):
        g = B.Grid(x, p)
        g.set_basis(basis)
        g.set_map_cache(cached)
        g.set_hamiltonian(ham)
        g.set_density(w)
        g.step(dt, 7)
        out.append(g.density())
        g.close()
    assert np.array_equal(out[0], out[1])

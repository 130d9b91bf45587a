"""Pins of the four-dimensional (2D2V) oracle, oracle/phase4d.py, against what
the method and the mathematics fix (Sec. "An Algorithm Based on Phase Space
Density Conservation": the same update in any dimension, with only Lambda and
Delta changing).  None re-types the oracle's formulas: they use the 2-D C
oracle on product states (independent code, itself pinned), quadrature of the
overlap integrals with a dense Kronecker solve, exact permutations, and
invariants."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from oracle import phase4d as P4
from paper_2007_12227_amd.inputs import H_FREE, H_PENDULUM, Axis, Hamiltonian, rng


def axes_small(nx=12, ny=10, npx=9, npy=11, pmax=2.5):
    return (Axis(-math.pi, math.pi, nx, True), Axis(-math.pi, math.pi, ny, True),
            Axis(-pmax, pmax, npx, False), Axis(-pmax, pmax, npy, False))


def bump(ax, c, s):
    """A Gaussian along one axis, evaluated at the nodes (wrapped on a periodic axis)."""
    z = ax.nodes() - c
    if ax.periodic:
        L = ax.hi - ax.lo
        z = (z + 0.5 * L) % L - 0.5 * L
    return np.exp(-z * z / (2 * s * s))


def outer(w_xpx, w_ypy):
    """w[py][px][y][x] = w2[py][y] w1[px][x] for w1 = w_xpx [px][x], w2 = w_ypy [py][y]."""
    return np.einsum("mk,li->mlki", w_ypy, w_xpx)


# ---- the separable case is the tensor product of two 2-D steps ----

@pytest.mark.parametrize("kind", [H_FREE, H_PENDULUM])
def test_separable_step_is_product_of_planar_steps(kind):
    """With V = -a cos x - b cos y the map is a product of two planar maps, Delta
    and Lambda factor over the planes, so a product state w1 (x) w2 advances as
    (2-D step of w1) (x) (2-D step of w2): the C oracle, pinned on its own."""
    x, y, px, py = axes_small()
    g = rng(80)
    w1 = g.uniform(0.1, 1.0, (px.n, x.n)) * bump(px, 0.3, 0.8)[:, None]
    w2 = g.uniform(0.1, 1.0, (py.n, y.n)) * bump(py, -0.2, 0.7)[:, None]
    a, b, dt, steps = 1.2, 0.7, 0.3, 3
    ham4 = P4.Ham4(P4.H4_FREE if kind == H_FREE else P4.H4_POTENTIAL, a=a, b=b, c=0.0)
    got = P4.run((x, y, px, py), ham4, outer(w1, w2), dt, steps)
    r1 = oracle.run(x, px, Hamiltonian(kind, a=a), w1, dt, steps).w
    r2 = oracle.run(y, py, Hamiltonian(kind, a=b), w2, dt, steps).w
    np.testing.assert_allclose(got, outer(r1, r2), atol=1e-13, rtol=0)


# ---- quadrature of eqs. 8-9 and a dense solve of eq. 10 ----

def test_step_equals_dense_update_by_quadrature():
    """On a 4 x 5 x 4 x 4 lattice: Delta from piecewise-exact quadrature of the
    1-D tent overlaps (a product of tents integrates as the product of its
    factors' integrals), Lambda the Kronecker product of the per-axis
    quadrature mass matrices, w_fin by a dense solve; random displacements up
    to 2.5 cells per axis, wrapping on the periodic axes."""
    x, y = Axis(-1.0, 1.0, 4, True), Axis(0.0, 2.0, 5, True)
    px, py = Axis(-1.0, 1.0, 4, False), Axis(-2.0, 1.0, 4, False)
    axes = (x, y, px, py)
    g = rng(81)
    shape = (py.n, px.n, y.n, x.n)
    w = g.uniform(-0.5, 1.0, shape)
    disp = tuple(g.uniform(-2.5, 2.5, shape) for _ in range(4))  # cells along x, y, px, py
    # Delta, row k = node k (flattened [py][px][y][x]), columns the lattice nodes
    n = w.size
    D = np.zeros((n, n))
    for k, (m, l, j, i) in enumerate(np.ndindex(*shape)):
        pos = [(x, i, 0), (y, j, 1), (px, l, 2), (py, m, 3)]
        ov = [np.array([brute.overlap_axis(ax, ax.lo + (idx + disp[a][m, l, j, i]) * ax.h, q)
                        for q in range(ax.n)]) for ax, idx, a in pos]
        D[k] = np.kron(np.kron(np.kron(ov[3], ov[2]), ov[1]), ov[0])
    lam1 = [np.array([[brute.overlap_axis(ax, ax.lo + a * ax.h, q) for q in range(ax.n)] for a in range(ax.n)])
            for ax in axes]
    lam = np.kron(np.kron(np.kron(lam1[3], lam1[2]), lam1[1]), lam1[0])
    cell = x.h * y.h * px.h * py.h
    b_ref = (D.T @ w.reshape(-1)) / cell
    np.testing.assert_allclose(P4.deposit(axes, disp, w).reshape(-1), b_ref, atol=1e-13, rtol=0)
    ref = np.linalg.solve(lam, D.T @ w.reshape(-1)).reshape(shape)
    np.testing.assert_allclose(P4.step(axes, P4.Ham4(P4.H4_FREE), 0.0, w, disp), ref, atol=1e-12, rtol=0)


def test_b3_is_the_tent_overlap():
    g = rng(82)
    for _ in range(100):
        h = g.uniform(0.2, 2.0)
        a, b = g.uniform(-3, 3, 2)
        assert brute.overlap(a, b, h) == pytest.approx(h * float(P4.b3((a - b) / h)), abs=1e-13)


# ---- exact special cases: permutations ----

def test_zero_motion_is_identity_including_open_edges():
    axes = axes_small(8, 6, 5, 7)
    w = rng(83).uniform(-1, 1, (7, 5, 6, 8))
    got = P4.run(axes, P4.Ham4(P4.H4_POTENTIAL, a=1.0, b=0.5, c=0.3), w, 0.0, 3)
    np.testing.assert_allclose(got, w, atol=1e-13, rtol=0)


def test_free_streaming_by_whole_cells_is_a_roll():
    """h_x = h_px = 1 and dt = 1: row (p_x, p_y) moves by (p_x, p_y) whole cells a step."""
    K = 3
    x, y = Axis(0.0, 12.0, 12, True), Axis(0.0, 10.0, 10, True)
    px, py = Axis(-K, K, 2 * K + 1, False), Axis(-2.0, 2.0, 5, False)  # integer momenta
    w = rng(84).uniform(-1, 1, (py.n, px.n, y.n, x.n))
    got = P4.run((x, y, px, py), P4.Ham4(P4.H4_FREE), w, 1.0, 2)
    ref = np.empty_like(w)
    for m, pyv in enumerate(py.nodes()):
        for l, pxv in enumerate(px.nodes()):
            ref[m, l] = np.roll(np.roll(w[m, l], int(2 * pxv), axis=1), int(2 * pyv), axis=0)
    np.testing.assert_allclose(got, ref, atol=1e-12, rtol=0)


# ---- invariants of the coupled map ----

def coupled_start(axes, seed=85):
    x, y, px, py = axes
    g = rng(seed)
    return (bump(py, 0.1, 0.35)[:, None, None, None] * bump(px, -0.2, 0.35)[None, :, None, None]
            * bump(y, 0.5, 0.8)[None, None, :, None] * bump(x, -0.4, 0.9)[None, None, None, :]
            * g.uniform(0.5, 1.0, (py.n, px.n, y.n, x.n)))


def test_sum_conserved_with_coupling_while_interior():
    """Partition of unity of the taps and 1^T M = 1^T on the periodic axes: the
    sum of the weights is kept while the density stays clear of the open
    momentum edges (eqs. 11-12): the inverse mass matrix decays by 2 - sqrt 3
    per node, so "clear" means some 25 nodes in FP64."""
    axes = axes_small(6, 6, 56, 54, pmax=3.0)
    x, y, px, py = axes
    w = (bump(py, 0.1, 0.25)[:, None, None, None] * bump(px, -0.1, 0.25)[None, :, None, None]
         * bump(y, 0.5, 0.8)[None, None, :, None] * bump(x, -0.4, 0.9)[None, None, None, :]
         * rng(85).uniform(0.5, 1.0, (py.n, px.n, y.n, x.n)))
    got = P4.run(axes, P4.Ham4(P4.H4_POTENTIAL, a=0.6, b=0.4, c=0.3), w, 0.1, 3)
    assert abs(got.sum() - w.sum()) <= 1e-13 * w.sum()


def test_linearity_and_point_reflection_with_coupling():
    """The step is linear in w for a static map, and V(-x,-y) = V(x,y) makes the
    map commute with (x, y, p) -> (-x, -y, -p): node i -> (n - i) mod n on a
    periodic axis centred at 0, j -> n - 1 - j on a symmetric open axis."""
    axes = axes_small(10, 8, 7, 9)
    ham = P4.Ham4(P4.H4_POTENTIAL, a=0.9, b=0.6, c=0.4)
    g = rng(86)
    w1, w2 = g.uniform(-1, 1, (2, 9, 7, 8, 10))
    s = lambda w: P4.step(axes, ham, 0.2, w)  # noqa: E731
    np.testing.assert_allclose(s(2.0 * w1 - 3.0 * w2), 2.0 * s(w1) - 3.0 * s(w2), atol=1e-12, rtol=0)

    def reflect(w):
        w = np.roll(w[:, :, ::-1, ::-1], 1, axis=(2, 3))  # i -> (n - i) mod n on x and y
        return w[::-1, ::-1]                             # j -> n - 1 - j on the momenta
    np.testing.assert_allclose(s(reflect(w1)), reflect(s(w1)), atol=1e-12, rtol=0)


# ---- diagnostics ----

def test_moments_of_a_product_state():
    """For w = w1 (x) w2 and c = 0, mass and energy are the planar ones combined
    (M = M1 M2, E = E1 M2 + M1 E2: the C oracle's moments, pinned by
    quadrature); the coupling term is checked by 1-D quadrature through
    cos(x - y) = cos x cos y + sin x sin y."""
    x, y, px, py = axes_small()
    g = rng(87)
    w1 = g.uniform(0.0, 1.0, (px.n, x.n))
    w2 = g.uniform(0.0, 1.0, (py.n, y.n))
    w = outer(w1, w2)
    a, b = 1.3, 0.8
    m4 = P4.moments((x, y, px, py), P4.Ham4(P4.H4_POTENTIAL, a=a, b=b), w)
    m1 = oracle.moments(x, px, Hamiltonian(H_PENDULUM, a=a), w1)
    m2 = oracle.moments(y, py, Hamiltonian(H_PENDULUM, a=b), w2)
    assert m4["mass"] == pytest.approx(m1["mass"] * m2["mass"], rel=1e-13)
    assert m4["energy"] == pytest.approx(m1["energy"] * m2["mass"] + m1["mass"] * m2["energy"], rel=1e-12)
    assert m4["mean_px"] == pytest.approx(m1["mean_p"], rel=1e-12)
    assert m4["mean_py"] == pytest.approx(m2["mean_p"], rel=1e-12)

    # the coupling energy -c int cos(x - y) f, by Simpson quadrature per axis
    c = 0.7
    m4c = P4.moments((x, y, px, py), P4.Ham4(P4.H4_POTENTIAL, a=a, b=b, c=c), w)

    def trig_integrals(ax, sub=240):
        t = np.linspace(ax.lo, ax.hi, ax.n * sub + 1)
        wt = np.ones_like(t)
        wt[1:-1:2], wt[2:-1:2] = 4, 2
        wt *= (ax.hi - ax.lo) / (ax.n * sub) / 3
        out = np.zeros((2, ax.n))
        for i in range(ax.n):
            tent = sum(brute.tent(t - (ax.lo + i * ax.h + k * (ax.hi - ax.lo)), ax.h) for k in (-1, 0, 1))
            out[0, i], out[1, i] = wt @ (np.cos(t) * tent), wt @ (np.sin(t) * tent)
        return out
    tx, ty = trig_integrals(x), trig_integrals(y)
    W = w.sum(axis=(0, 1))  # [y][x], summed over the momenta
    coupling = -c * px.h * py.h * (np.einsum("ki,i,k->", W, tx[0], ty[0]) + np.einsum("ki,i,k->", W, tx[1], ty[1]))
    assert m4c["energy"] - m4["energy"] == pytest.approx(coupling, rel=1e-10)


def test_entropy_closed_form():
    axes = axes_small(6, 5, 4, 4)
    w = np.full((4, 4, 5, 6), 2.0)
    m = P4.moments(axes, P4.Ham4(P4.H4_FREE), w)
    assert m["entropy"] == pytest.approx(-m["mass"] * math.log(2.0), rel=1e-13)


def test_push_is_second_order_against_an_ode_integrator():
    """The drift-kick-drift push against scipy's DOP853 on Hamilton's equations,
    the force taken as minus a central-difference gradient of V (independent of
    the push's own derivative): the one-step error falls ~8x per halving of dt
    (local error of a second-order method), for the coupled potential."""
    from scipy.integrate import solve_ivp
    axes = axes_small(5, 4, 3, 3, pmax=1.5)
    a, b, c = 0.9, 0.5, 0.7
    ham = P4.Ham4(P4.H4_POTENTIAL, a=a, b=b, c=c)
    V = lambda x, y: -a * np.cos(x) - b * np.cos(y) - c * np.cos(x - y)  # noqa: E731
    e = 1e-6

    def rhs(_, z):
        x, y, px, py = z
        gx = (V(x + e, y) - V(x - e, y)) / (2 * e)
        gy = (V(x, y + e) - V(x, y - e)) / (2 * e)
        return [px, py, -gx, -gy]

    X, Y, PX, PY = P4.lattice(axes)
    errs = []
    for dt in (0.2, 0.1, 0.05):
        d = P4.push(axes, ham, dt)
        err = 0.0
        for idx in np.ndindex(*X.shape):
            z0 = [X[idx], Y[idx], PX[idx], PY[idx]]
            z1 = solve_ivp(rhs, (0, dt), z0, method="DOP853", rtol=1e-12, atol=1e-12).y[:, -1]
            got = [z0[k] + d[k][idx] * axes[k].h for k in range(4)]
            err = max(err, max(abs(got[k] - z1[k]) for k in range(4)))
        errs.append(err)
    assert errs[0] / errs[1] > 6 and errs[1] / errs[2] > 6, errs

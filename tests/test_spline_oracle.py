"""Pins of the B-spline basis oracle (oracle/spline_basis.py) against what the
mathematics fixes, independently of its closed-form taps: the basis function
is retyped here from its piecewise definition, overlaps are integrated by
Gauss-Legendre quadrature (exact on each polynomial piece), the Fourier gain
comes from the B-spline's transform by Poisson summation, and the invariants
(mass on a periodic lattice, lattice-aligned motion) hold at any size."""
import math

import numpy as np
import pytest

import oracle
from oracle import spline_basis as Q
from paper_2007_12227_amd.inputs import H_FEL, H_PENDULUM, H_SHO_EXACT, Axis, Hamiltonian, fel_gaussian, rng

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

_GL_X, _GL_W = np.polynomial.legendre.leggauss(4)  # exact to degree 7


def b2(s: float) -> float:
    """Quadratic B-spline, piece by piece."""
    s = abs(s)
    if s < 0.5:
        return 0.75 - s * s
    if s < 1.5:
        return 0.5 * (1.5 - s) ** 2
    return 0.0


def basis(degree):
    """The basis function of unit width: the quadratic spline retyped above, or
    the tent oracle's cubic spline (written independently in C)."""
    return b2 if degree == 2 else oracle.b3


def overlap(a: float, b: float, h: float, degree: int = 2) -> float:
    """int_R Bd((t-a)/h) Bd((t-b)/h) dt, quadrature on every interval between
    the two functions' knots (the product is a polynomial of degree 2d there)."""
    if abs(a - b) >= (degree + 1) * h:
        return 0.0
    f = basis(degree)
    offs = [k - 0.5 * (degree + 1) for k in range(degree + 2)]
    knots = sorted({a + k * h for k in offs} | {b + k * h for k in offs})
    total = 0.0
    for lo, hi in zip(knots[:-1], knots[1:]):
        if hi <= lo:
            continue
        mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
        for xg, wg in zip(_GL_X, _GL_W):
            t = mid + half * xg
            total += half * wg * f((t - a) / h) * f((t - b) / h)
    return total


def overlap_axis(axis, centre: float, j: int, degree: int = 2) -> float:
    xj = axis.lo + j * axis.h
    if not axis.periodic:
        return overlap(centre, xj, axis.h, degree)
    L = axis.hi - axis.lo
    return sum(overlap(centre, xj + m * L, axis.h, degree) for m in range(-2, 3))


def dense_step(x, p, du, dv, w, degree=2):
    """Lambda^{-1} Delta^T w (eq. 10) with Lambda and Delta from quadrature."""
    Lx = np.array([[overlap_axis(x, x.lo + a * x.h, b, degree) for b in range(x.n)] for a in range(x.n)])
    Lp = np.array([[overlap_axis(p, p.lo + a * p.h, b, degree) for b in range(p.n)] for a in range(p.n)])
    D = np.zeros((x.n * p.n, x.n * p.n))
    for jk in range(p.n):
        for ik in range(x.n):
            X = x.lo + (ik + du[jk, ik]) * x.h
            P = p.lo + (jk + dv[jk, ik]) * p.h
            ox = np.array([overlap_axis(x, X, b, degree) for b in range(x.n)])
            op = np.array([overlap_axis(p, P, b, degree) for b in range(p.n)])
            D[jk * x.n + ik] = np.kron(op, ox)
    b = D.T @ w.reshape(-1)
    return b, np.linalg.solve(np.kron(Lp, Lx), b).reshape(p.n, x.n)


def test_bspline_low_degrees_are_the_textbook_ones():
    s = np.linspace(-3.2, 3.2, 257)
    assert np.allclose(Q.bspline(1, s), np.maximum(0.0, 1.0 - np.abs(s)), atol=1e-15)
    assert np.allclose(Q.bspline(2, s), [b2(t) for t in s], atol=1e-15)
    # the tent oracle's cubic, written independently in C
    assert np.allclose(Q.bspline(3, s), [oracle.b3(t) for t in s], atol=1e-15)


def test_overlap_of_quadratic_splines_is_quintic_spline():
    """The overlap of two quadratic B-splines d cells apart is h B5(d)
    (B5 = B2 * B2 * ... the six-fold box convolution), and at the integer
    offsets B5 = 1/120, 26/120, 66/120."""
    h = 0.37
    for d in np.linspace(-3.3, 3.3, 67):
        assert abs(overlap(0.0, d * h, h) - h * float(Q.bspline(5, d))) <= 1e-14
    assert np.allclose(Q.bspline(5, np.arange(-3, 4)), np.array([0, 1, 26, 66, 26, 1, 0]) / 120.0,
                       atol=1e-16)


def test_overlap_of_cubic_splines_is_septic_spline():
    """Cubic basis: the overlap is h B7(d) (quadrature of the C oracle's cubic),
    and B7 at the integers is [1, 120, 1191, 2416, 1191, 120, 1]/5040."""
    h = 0.29
    for d in np.linspace(-4.3, 4.3, 87):
        assert abs(overlap(0.0, d * h, h, 3) - h * float(Q.bspline(7, d))) <= 5e-14
    assert np.allclose(Q.bspline(7, np.arange(-4, 5)),
                       np.array([0, 1, 120, 1191, 2416, 1191, 120, 1, 0]) / 5040.0, atol=1e-15)


@pytest.mark.parametrize("degree", [2, 3])
@pytest.mark.parametrize("px,pp", [(True, False), (False, False), (True, True)])
def test_deposit_and_step_match_quadrature(px, pp, degree):
    """Deposit = Delta^T w and the full step = Lambda^{-1} Delta^T w, Delta and
    Lambda integrated from the basis functions (eqs. 8-10), on 9 x 7 nodes
    with displacements up to 3 cells, so taps wrap and fall past open edges."""
    x = Axis(-1.0, 1.7, 9, px)
    p = Axis(-0.8, 1.1, 7, pp)
    r = rng(901)
    du = r.uniform(-3.0, 3.0, (p.n, x.n))
    dv = r.uniform(-3.0, 3.0, (p.n, x.n))
    w = r.random((p.n, x.n)) - 0.3
    b_ref, w_ref = dense_step(x, p, du, dv, w, degree)
    b = Q.deposit(x, p, du, dv, w, degree) * x.h * p.h
    assert np.allclose(b.reshape(-1), b_ref, rtol=0, atol=1e-13)
    got = Q.step(x, p, du, dv, w, degree)
    assert np.abs(got - w_ref).max() <= 1e-11 * np.abs(w_ref).max()


@pytest.mark.parametrize("degree", [2, 3])
@pytest.mark.parametrize("n,periodic", [(5, True), (12, True), (5, False), (13, False)])
def test_mass_line_is_the_overlap_matrix(n, periodic, degree):
    ax = Axis(0.0, 1.0, n, periodic)
    ref = np.array([[overlap_axis(ax, ax.lo + a * ax.h, b, degree) for b in range(n)] for a in range(n)]) / ax.h
    assert np.allclose(Q.mass_line(n, periodic, degree), ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("degree", [2, 3])
def test_sum_conserved_on_periodic_lattice(degree):
    """Constants lie in the span of the basis on a periodic lattice, so the L2
    projection keeps the integral: sum w is conserved for any motion."""
    x = Axis(0.0, 1.0, 40, True)
    p = Axis(0.0, 2.0, 24, True)
    r = rng(902)
    w = r.random((p.n, x.n))
    du = r.normal(0, 1.5, (p.n, x.n))
    dv = r.normal(0, 1.5, (p.n, x.n))
    got = Q.step(x, p, du, dv, w, degree)
    assert abs(got.sum() - w.sum()) <= 1e-12 * w.sum()


@pytest.mark.parametrize("degree", [2, 3])
def test_integer_shift_is_a_rotation_and_zero_motion_identity(degree):
    """A density moved by whole cells stays in the span: the step returns it
    shifted exactly; no motion returns it unchanged, open edges included."""
    x = Axis(-math.pi, math.pi, 32, True)
    p = Axis(-3.0, 3.0, 21, False)
    w = rng(903).random((p.n, x.n))
    du = np.repeat(np.arange(p.n)[:, None] - 10, x.n, axis=1).astype(np.float64)
    dv = np.zeros_like(du)
    got = Q.step(x, p, du, dv, w, degree)
    for j in range(p.n):
        assert np.allclose(got[j], np.roll(w[j], j - 10), rtol=0, atol=1e-12)
    assert np.allclose(Q.step(x, p, 0 * du, dv, w, degree), w, rtol=0, atol=1e-12)


@pytest.mark.parametrize("degree", [2, 3])
def test_fourier_gain_from_the_spline_transform(degree):
    """A uniform shift a of a Fourier mode exp(i theta j) multiplies it by
    G = sum_k Bh(2 pi k - theta) e^{i (2 pi k - theta) a} / sum_k Bh(2 pi k - theta),
    Bh(w) = (sin(w/2) / (w/2))^6 the quintic B-spline's transform (Poisson
    summation over the lattice)."""
    n = 48
    x = Axis(0.0, 1.0, n, True)
    p = Axis(0.0, 1.0, 6, True)
    j = np.arange(n)
    k = np.arange(-200, 201)

    def bh(om):
        return np.where(om == 0, 1.0, np.sinc(om / (2 * np.pi)) ** (2 * degree + 2))

    for m, a in ((1, 0.3), (5, 0.71), (11, -0.45), (23, 0.5)):
        theta = 2 * np.pi * m / n
        om = 2 * np.pi * k - theta
        G = (bh(om) * np.exp(1j * om * a)).sum() / bh(om).sum()
        for part, wj in ((np.real, np.cos(theta * j)), (np.imag, np.sin(theta * j))):
            w = np.repeat(wj[None, :], p.n, axis=0)
            du = np.full((p.n, n), a)
            got = Q.step(x, p, du, 0 * du, w, degree)
            exp = part(G * np.exp(1j * theta * j))
            assert np.allclose(got, exp[None, :], rtol=0, atol=1e-12), (m, a)
        # the projection damps but never amplifies
        assert abs(G) <= 1.0 + 1e-15


def test_quadratic_basis_transports_smooth_data_more_accurately_than_tents():
    """One revolution of the exact rotation on 64^2 nodes in 32 steps: the
    smoother basis lands closer to the start than the tent oracle."""
    x = Axis(-6.0, 6.0, 64, False)
    p = Axis(-6.0, 6.0, 64, False)
    X, P = np.meshgrid(x.nodes(), p.nodes())
    w0 = np.exp(-((X - 1.5) ** 2 + P ** 2) / (2 * 0.8 ** 2))
    ham = Hamiltonian(H_SHO_EXACT, omega=1.0)
    dt = 2 * np.pi / 32
    quad = Q.run(x, p, ham, w0, dt, 32)
    tent = oracle.run(x, p, ham, w0, dt, 32).w
    e_quad, e_tent = oracle.rel_l1(quad, w0), oracle.rel_l1(tent, w0)
    assert e_quad < 0.5 * e_tent, (e_quad, e_tent)


def test_pendulum_run_conserves_mass_away_from_the_edges():
    """Support well inside the open momentum range (the inverse mass matrix
    rings out at about 0.43 per cell, so the edges need room)."""
    x = Axis(-math.pi, math.pi, 48, True)
    p = Axis(-5.0, 5.0, 64, False)
    X, P = np.meshgrid(x.nodes(), p.nodes())
    w0 = np.exp(-(X ** 2 + P ** 2) / (2 * 0.5 ** 2))
    w = Q.run(x, p, Hamiltonian(H_PENDULUM, a=1.0), w0, 0.1, 20)
    assert abs(w.sum() - w0.sum()) <= 1e-10 * w0.sum()


@pytest.mark.parametrize("degree", [2, 3])
@pytest.mark.parametrize("kind", [H_PENDULUM, H_SHO_EXACT])
def test_moments_are_integrals_of_the_expansion(kind, degree):
    """Mass and energy of f = sum w_j B2 B2 on 9 x 7 nodes against quadrature
    of f itself (per axis: every polynomial piece of each basis function)."""
    if kind == H_PENDULUM:
        x, p = Axis(-math.pi, math.pi, 9, True), Axis(-2.0, 2.0, 7, False)
        ham = Hamiltonian(kind, a=1.3)
    else:
        x, p = Axis(-2.0, 2.5, 9, False), Axis(-2.0, 2.0, 7, False)
        ham = Hamiltonian(kind, omega=1.0)
    w = rng(904).random((p.n, x.n)) - 0.2

    f = basis(degree)

    def integral(axis, j, g):
        c = axis.lo + j * axis.h
        total = 0.0
        for k in range(degree + 1):
            lo = c + (k - 0.5 * (degree + 1)) * axis.h
            mid, half = lo + 0.5 * axis.h, 0.5 * axis.h
            for xg, wg in zip(*np.polynomial.legendre.leggauss(12)):
                t = mid + half * xg
                total += half * wg * f((t - c) / axis.h) * g(t)
        return total

    one_x = np.array([integral(x, i, lambda t: 1.0) for i in range(x.n)])
    one_p = np.array([integral(p, j, lambda t: 1.0) for j in range(p.n)])
    p2 = np.array([integral(p, j, lambda t: 0.5 * t * t) for j in range(p.n)])
    if kind == H_PENDULUM:
        vx = np.array([integral(x, i, lambda t: -ham.a * math.cos(t)) for i in range(x.n)])
    else:
        vx = np.array([integral(x, i, lambda t: 0.5 * t * t) for i in range(x.n)])
    mass = float((w * np.outer(one_p, one_x)).sum())
    energy = float((w * (np.outer(p2, one_x) + np.outer(one_p, vx))).sum())
    m = Q.moments(x, p, ham, w, degree)
    assert abs(m["mass"] - mass) <= 1e-13
    assert abs(m["energy"] - energy) <= 1e-12 * abs(energy)


@pytest.mark.parametrize("degree", [2, 3])
@pytest.mark.parametrize("delta,sigma2", [(0.0, 0.0), (0.3, 0.4)])
def test_fel_invariant_is_conserved_with_spline_basis(delta, sigma2, degree):
    """|A|^2 + N0^-1 sum w eta is conserved by the exact-kick step and the
    projection: linear functions lie in the span of the quadratic splines too
    (they reproduce polynomials of degree 2), and the nodal sum of w eta is
    the integral of eta f over the expansion (each spline is symmetric), so
    the projection keeps it while the beam is clear of the energy edges."""
    inst = fel_gaussian(64, 1, npp=128)
    ham = Hamiltonian(H_FEL, A_re=2e-2, A_im=-1e-2, fel_delta=delta, fel_sigma2=sigma2)
    eta = inst.p.nodes()[:, None]
    N0 = float(inst.w0.sum())
    e0 = abs(complex(ham.A_re, ham.A_im)) ** 2 + float((inst.w0 * eta).sum()) / N0
    w, A = Q.run_fel(inst.x, inst.p, ham, inst.w0, 0.05, 40, degree=degree)
    e1 = abs(A) ** 2 + float((w * eta).sum()) / N0
    assert abs(e1 - e0) <= 1e-12, (e0, e1)
    assert abs(A - complex(ham.A_re, ham.A_im)) > 1e-4  # the field did move

"""FP64 oracle of the method with B-spline basis functions of degree d = 2
(quadratic) or 3 (cubic) (test infrastructure: only the tests use it; the
product library does not).

The paper expands the density in tents (eq. 4) and builds the update from
the basis functions' overlaps (eqs. 8-10); smoother local basis functions are
the extension its discussion points to.  Here the basis function of a node is
the centred B-spline of degree d and width (d + 1) h, Bd((x - x_j) / h).  The
overlap of two of them whose centres are s h apart is h B(2d+1)(s), so with
this basis:
  * Delta (eq. 9): a node moved to u (in cells) gives weight B(2d+1)(u - c) to
    the 2d + 2 nodes c = floor(u) - d .. floor(u) + d + 1 of each axis;
  * Lambda (eq. 8) = h_x h_p M_x (x) M_p, M the values of B(2d+1) at the
    integer offsets -d .. d ([1, 26, 66, 26, 1] / 120 for d = 2), cyclic on a
    periodic axis and truncated on an open one (full basis functions at the
    edge nodes; weight moved past an edge is lost, as with tents);
  * the update is w_fin = Lambda^{-1} Delta^T w (eq. 10), the push being the
    tent oracle's (it does not depend on the basis).
(d = 1 is the tent basis itself.)  Every step here is written out plainly
(numpy scatter, dense per-axis solves) and is meant for lattices of a few
hundred nodes per axis.
"""
from __future__ import annotations

import math

import numpy as np

from . import push as _push

H_SHO_EXACT, H_PENDULUM = 1, 2


def bspline(k: int, s) -> np.ndarray:
    """Centred cardinal B-spline of degree k (support [-(k+1)/2, (k+1)/2]):
    B_k(s) = 1/k! sum_j (-1)^j C(k+1, j) (s + (k+1)/2 - j)_+^k."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    for j in range(k + 2):
        out += (-1) ** j * math.comb(k + 1, j) * np.maximum(s + 0.5 * (k + 1) - j, 0.0) ** k
    out /= math.factorial(k)
    # the sum cancels to rounding outside the support: make it exact there
    return np.where(np.abs(s) < 0.5 * (k + 1), out, 0.0)


def taps(u, degree: int = 2) -> tuple[np.ndarray, np.ndarray]:
    """First tap cell floor(u) - d and the 2d + 2 weights B(2d+1)(u - c)."""
    u = np.asarray(u, dtype=np.float64)
    k0 = np.floor(u).astype(np.int64) - degree
    c = k0[..., None] + np.arange(2 * degree + 2)
    return k0, bspline(2 * degree + 1, u[..., None] - c)


def deposit(x, p, du, dv, w, degree: int = 2) -> np.ndarray:
    """b = Delta^T w / (h_x h_p) for nodes moved by (du, dv) cells."""
    n_p, n_x = p.n, x.n
    ntaps = 2 * degree + 2
    jj, ii = np.meshgrid(np.arange(n_p), np.arange(n_x), indexing="ij")
    kx, bx = taps(ii + np.asarray(du, dtype=np.float64), degree)
    kp, bp = taps(jj + np.asarray(dv, dtype=np.float64), degree)
    b = np.zeros((n_p, n_x))
    w = np.asarray(w, dtype=np.float64)
    for q in range(ntaps):
        rows = kp + q
        rows = np.mod(rows, n_p) if p.periodic else rows
        for r in range(ntaps):
            cols = kx + r
            cols = np.mod(cols, n_x) if x.periodic else cols
            # on an open axis, taps past the edge nodes are dropped
            keep = (rows >= 0) & (rows < n_p) & (cols >= 0) & (cols < n_x)
            np.add.at(b, (rows[keep], cols[keep]), (w * bp[..., q] * bx[..., r])[keep])
    return b


def mass_line(n: int, periodic: bool, degree: int = 2) -> np.ndarray:
    """M along one axis: B(2d+1) at the integer offsets, wrapped on a periodic axis."""
    M = np.zeros((n, n))
    for a in range(n):
        for d in range(-degree, degree + 1):
            bval = float(bspline(2 * degree + 1, d))
            if periodic:
                M[a, (a + d) % n] += bval
            elif 0 <= a + d < n:
                M[a, a + d] += bval
    return M


def solve(x, p, b, degree: int = 2) -> np.ndarray:
    """(M_x^{-1} (x) M_p^{-1}) b: dense solves along each axis."""
    b = np.asarray(b, dtype=np.float64)
    y = np.linalg.solve(mass_line(x.n, x.periodic, degree), b.T).T
    return np.linalg.solve(mass_line(p.n, p.periodic, degree), y)


def step(x, p, du, dv, w, degree: int = 2) -> np.ndarray:
    return solve(x, p, deposit(x, p, du, dv, w, degree), degree)


def run(x, p, ham, w0, dt, steps, degree: int = 2) -> np.ndarray:
    """``steps`` steps of a Hamiltonian whose push does not depend on the
    state (free streaming, the exact rotation, the pendulum)."""
    du, dv = _push(x, p, ham, dt)
    w = np.array(w0, dtype=np.float64, copy=True)
    for _ in range(int(steps)):
        w = step(x, p, du, dv, w, degree)
    return w


FEL_RK4 = 1


def run_fel(x, p, ham, w0, dz, steps, A0=None, N0=None, degree: int = 2):
    """``steps`` steps of the 1-D FEL (eqs. 13a-c), the push as the tent oracle
    takes it (it does not depend on the basis), then the projection onto this
    basis.  Drift-kick-drift with the kick integrated exactly: the bunching
    b = N0^-1 sum w e^{-i psi} of the state at its half-drift phases, the kick
    in the field A + b dz/2 + i sigma2 b, then A += b dz.  Runge-Kutta
    (ham.integrator == FEL_RK4): the nodes as particles of charge w, and A,
    advanced by the classical fourth-order method.  Returns (w, A)."""
    from . import bunching as _bunching
    from . import push_rk4 as _push_rk4
    w = np.array(w0, dtype=np.float64, copy=True)
    A = complex(ham.A_re, ham.A_im) if A0 is None else complex(A0)
    N0 = float(w.sum()) if N0 is None else float(N0)
    for _ in range(int(steps)):
        if getattr(ham, "integrator", 0) == FEL_RK4:
            du, dv, A = _push_rk4(x, p, ham, dz, w, N0, A)
        else:
            bn = _bunching(x, p, ham, dz, w, N0)
            At = A + 0.5 * dz * bn + 1j * ham.fel_sigma2 * bn
            du, dv = _push(x, p, ham, dz, np.array([At.real, At.imag]))
            A += dz * bn
        w = step(x, p, du, dv, w, degree)
    return w, A


def moments(x, p, ham, w, degree: int = 2) -> dict:
    """Diagnostics of f = sum_j w_j Bd((x - x_j)/h_x) Bd((p - p_j)/h_p), the C
    oracle's quantities with this basis: every basis function integrates to
    h, its second moment about its centre is h^3 (d + 1)/12 (d + 1 unit boxes
    convolved, each of variance 1/12), and its integral against cos x is
    h sinc(h/2)^(d+1) cos x_j (the transform of a box is a sinc).  The
    entropy and the negative mass are sums over the weights, as for tents."""
    w = np.asarray(w, dtype=np.float64)
    cell = x.h * p.h
    var = (degree + 1) / 12.0
    X, P = np.meshgrid(x.nodes(), p.nodes())
    e = 0.5 * (P ** 2 + var * p.h ** 2)
    if ham.kind == H_PENDULUM:
        y = 0.5 * x.h
        e = e - ham.a * (math.sin(y) / y) ** (degree + 1) * np.cos(X)
    elif ham.kind == H_SHO_EXACT:
        e = e + 0.5 * (X ** 2 + var * x.h ** 2)
    pos = w > 0
    return {
        "sum_w": float(w.sum()),
        "mass": cell * float(w.sum()),
        "neg_mass": -cell * float(w[w < 0].sum()),
        "l1": cell * float(np.abs(w).sum()),
        "entropy": -cell * float((w[pos] * np.log(w[pos])).sum()),
        "mean_p": float((w * P).sum() / w.sum()) if w.sum() != 0 else 0.0,
        "energy": cell * float((w * e).sum()),
    }

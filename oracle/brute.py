"""Brute-force checks for tiny grids (test infrastructure).

Builds the paper's matrices straight from their integral definitions
(Sec. Algorithm, eqs. 8-9) by exact piecewise quadrature of tent products,
then applies the update of eq. 10 with a dense solve.  Nothing here uses the
closed-form B-spline taps or the banded solves of ``vp_oracle.c``, so it pins
them independently.  Only meant for grids of a few hundred nodes.
"""
from __future__ import annotations

import numpy as np


def tent(s: np.ndarray, h: float) -> np.ndarray:
    return np.maximum(0.0, 1.0 - np.abs(s) / h)


def overlap(a: float, b: float, h: float) -> float:
    """int_R tent(x-a) tent(x-b) dx, exact: Simpson's rule on every interval
    between breakpoints, where the integrand is a quadratic polynomial."""
    if abs(a - b) >= 2.0 * h:
        return 0.0
    pts = sorted({a - h, a, a + h, b - h, b, b + h})

    def f(x: float) -> float:
        return max(0.0, 1.0 - abs(x - a) / h) * max(0.0, 1.0 - abs(x - b) / h)

    total = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        if hi > lo:
            total += (hi - lo) / 6.0 * (f(lo) + 4.0 * f(0.5 * (lo + hi)) + f(hi))
    return total


def overlap_axis(axis, centre: float, j: int) -> float:
    """Overlap of a tent at ``centre`` with the tent of lattice node j; on a
    periodic axis the tent of node j is summed over its periodic images."""
    xj = axis.lo + j * axis.h
    if not axis.periodic:
        return overlap(centre, xj, axis.h)
    L = axis.hi - axis.lo
    total = 0.0
    for m in range(-3, 4):
        total += overlap(centre, xj + m * L, axis.h)
    return total


def mass_matrix(x, p) -> np.ndarray:
    """Lambda_{jj'} (eq. 8) over the flattened lattice k = j_p * n_x + i_x."""
    Lx = np.array([[overlap_axis(x, x.lo + a * x.h, b) for b in range(x.n)] for a in range(x.n)])
    Lp = np.array([[overlap_axis(p, p.lo + a * p.h, b) for b in range(p.n)] for a in range(p.n)])
    return np.kron(Lp, Lx)


def transfer_matrix(x, p, dx: np.ndarray, dp: np.ndarray) -> np.ndarray:
    """Delta_{kj'} (eq. 9): overlap of the tent of node k moved by (dx_k, dp_k)
    with the tent of node j'.  dx, dp are in physical units, shape [n_p][n_x]."""
    n = x.n * p.n
    D = np.zeros((n, n))
    for jk in range(p.n):
        for ik in range(x.n):
            k = jk * x.n + ik
            X = x.lo + ik * x.h + dx[jk, ik]
            P = p.lo + jk * p.h + dp[jk, ik]
            ox = np.array([overlap_axis(x, X, b) for b in range(x.n)])
            op = np.array([overlap_axis(p, P, b) for b in range(p.n)])
            D[k, :] = np.kron(op, ox)
    return D


def step_dense(x, p, dx: np.ndarray, dp: np.ndarray, w: np.ndarray) -> np.ndarray:
    """w_fin = Lambda^{-1} Delta^T w_in (eq. 10) with a dense solve."""
    lam = mass_matrix(x, p)
    D = transfer_matrix(x, p, dx, dp)
    return np.linalg.solve(lam, D.T @ w.reshape(-1)).reshape(p.n, x.n)

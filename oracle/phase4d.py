"""FP64 oracle of the method on a four-dimensional phase space (x, y, p_x, p_y).

TEST INFRASTRUCTURE.  Only the tests, the GPU smoke check and the CPU-baseline
leg of the benchmark use this module; the product library never does, and it
shares no code with it.

The paper's closing remark on the algorithm (Sec. "An Algorithm Based on
Phase Space Density Conservation") is that the method carries over to any
dimension with only Lambda and Delta changing.  With a tensor product of tents
on every axis, f = sum_j w_j prod_d Lambda(z_d - z_{j,d}) (eq. 4 in 2D2V), the
overlaps factor over the axes (Fubini):
    Delta_{kj'}  = prod_d h_d B3((Z_{k,d} - z_{j',d}) / h_d)          (eq. 9)
    Lambda_{jj'} = prod_d h_d M_d                                      (eq. 8)
with B3 the centred cubic B-spline (the overlap of two unit tents) and
M = tridiag(1/6, 2/3, 1/6), cyclic on a periodic axis.  So one step of
eq. 10 is a 4^4 = 256-tap scatter of every pushed node followed by
M_x^{-1} (x) M_y^{-1} (x) M_px^{-1} (x) M_py^{-1}, one dense inverse per axis
applied along that axis (a library primitive; the lattices here are small).

Arrays are [n_py][n_px][n_y][n_x] (x fastest); x and y are periodic, the
momenta open (full tents at the edge nodes, taps past an edge are lost: the
readings of the 2-D case, axis by axis).

Hamiltonians: free streaming, and H = |p|^2/2 + V(x, y) with
    V = -a cos x - b cos y - c cos(x - y)
(c = 0: two uncoupled pendulums; c != 0 couples the planes) advanced by the
drift-kick-drift leapfrog (drift dt/2, kick dt with the force -grad V at the
half-drift point, drift dt/2), the 2-D reading of the pendulum carried over.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

H4_FREE, H4_POTENTIAL = 0, 2


@dataclass(frozen=True)
class Ham4:
    kind: int
    a: float = 0.0
    b: float = 0.0
    c: float = 0.0


def b3(s):
    """Centred cubic B-spline: the overlap of two unit tents whose centres are
    s apart (the tent autocorrelation)."""
    s = np.abs(np.asarray(s, dtype=np.float64))
    return np.where(s < 1.0, 2.0 / 3.0 - s * s + 0.5 * s ** 3,
                    np.where(s < 2.0, (2.0 - s) ** 3 / 6.0, 0.0))


def lattice(axes):
    """Node coordinates, each broadcast to the array shape [py][px][y][x]."""
    x, y, px, py = axes
    PY, PX, Y, X = np.meshgrid(py.nodes(), px.nodes(), y.nodes(), x.nodes(), indexing="ij")
    return X, Y, PX, PY


def push(axes, ham: Ham4, dt: float):
    """Displacement of every node in cells along each axis: (du_x, du_y, du_px, du_py)."""
    x, y, px, py = axes
    X, Y, PX, PY = lattice(axes)
    if ham.kind == H4_FREE:
        return PX * dt / x.h, PY * dt / y.h, np.zeros_like(PX), np.zeros_like(PY)
    xh, yh = X + 0.5 * dt * PX, Y + 0.5 * dt * PY
    # force -grad V at the half-drift point
    fx = -(ham.a * np.sin(xh) + ham.c * np.sin(xh - yh))
    fy = -(ham.b * np.sin(yh) - ham.c * np.sin(xh - yh))
    pxn, pyn = PX + dt * fx, PY + dt * fy
    xn, yn = xh + 0.5 * dt * pxn, yh + 0.5 * dt * pyn
    return (xn - X) / x.h, (yn - Y) / y.h, (pxn - PX) / px.h, (pyn - PY) / py.h


def deposit(axes, disp, w):
    """b = Delta^T w / prod h: every node's weight times the product of the
    four B3 overlaps with the lattice nodes its moved tent reaches (cells
    floor(u) - 1 .. floor(u) + 2 per axis)."""
    shape = w.shape
    idx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")  # [py][px][y][x] indices
    # per axis (in array order py, px, y, x): the moved position in cells
    order = [(3, axes[3]), (2, axes[2]), (1, axes[1]), (0, axes[0])]
    u = [idx[k] + disp[a] for k, (a, _) in enumerate(order)]
    base = [np.floor(v).astype(np.int64) for v in u]
    b = np.zeros(w.size)
    for r in np.ndindex(4, 4, 4, 4):
        wt = w.astype(np.float64).copy()
        flat = np.zeros(w.shape, dtype=np.int64)
        keep = np.ones(w.shape, dtype=bool)
        stride = 1
        for k in (3, 2, 1, 0):  # x, y, px, py: array axes from the fastest
            ax = order[k][1]
            cell = base[k] + (r[k] - 1)
            wt = wt * b3(u[k] - cell)
            if ax.periodic:
                cell = np.mod(cell, ax.n)
            else:
                keep &= (cell >= 0) & (cell < ax.n)
                cell = np.clip(cell, 0, ax.n - 1)
            flat += cell * stride
            stride *= ax.n
        b += np.bincount(flat[keep], weights=wt[keep], minlength=w.size)
    return b.reshape(shape)


def mass_line(ax) -> np.ndarray:
    """M = tridiag(1/6, 2/3, 1/6) of one axis (eq. 8 per unit spacing),
    cyclic on a periodic axis, truncated on an open one."""
    n = ax.n
    M = np.diag(np.full(n, 2.0 / 3.0)) + np.diag(np.full(n - 1, 1.0 / 6.0), 1) + np.diag(np.full(n - 1, 1.0 / 6.0), -1)
    if ax.periodic:
        M[0, n - 1] += 1.0 / 6.0
        M[n - 1, 0] += 1.0 / 6.0
    return M


def solve(axes, b):
    """(M_x^{-1} (x) M_y^{-1} (x) M_px^{-1} (x) M_py^{-1}) b."""
    out = np.asarray(b, dtype=np.float64)
    for arr_axis, ax in ((3, axes[0]), (2, axes[1]), (1, axes[2]), (0, axes[3])):
        Minv = np.linalg.inv(mass_line(ax))
        out = np.moveaxis(np.tensordot(Minv, out, axes=([1], [arr_axis])), 0, arr_axis)
    return out


def step(axes, ham: Ham4, dt: float, w, disp=None):
    disp = push(axes, ham, dt) if disp is None else disp
    return solve(axes, deposit(axes, disp, w))


def run(axes, ham: Ham4, w0, dt: float, steps: int):
    w = np.array(w0, dtype=np.float64)
    disp = push(axes, ham, dt)  # the map does not depend on the state
    for _ in range(steps):
        w = step(axes, ham, dt, w, disp)
    return w


def moments(axes, ham: Ham4, w) -> dict:
    """Sums over the weights (the 2-D diagnostics, axis by axis): the integral
    of f is prod h sum w; energy integrates H over the tent expansion with the
    exact tent integrals int p^2 Lambda = h (p_j^2 + h^2/6) and
    int e^{i x} Lambda = h sinc^2(h/2) e^{i x_j}."""
    x, y, px, py = axes
    w = np.asarray(w, dtype=np.float64)
    cell = x.h * y.h * px.h * py.h
    X, Y, PX, PY = lattice(axes)
    sx, sy = (math.sin(0.5 * x.h) / (0.5 * x.h)) ** 2, (math.sin(0.5 * y.h) / (0.5 * y.h)) ** 2
    e = 0.5 * (PX ** 2 + px.h ** 2 / 6.0) + 0.5 * (PY ** 2 + py.h ** 2 / 6.0)
    if ham.kind == H4_POTENTIAL:
        e = e - ham.a * sx * np.cos(X) - ham.b * sy * np.cos(Y) - ham.c * sx * sy * np.cos(X - Y)
    pos = w > 0
    s = float(w.sum())
    return {"sum_w": s, "mass": cell * s, "neg_mass": -cell * float(w[w < 0].sum()),
            "l1": cell * float(np.abs(w).sum()), "entropy": -cell * float((w[pos] * np.log(w[pos])).sum()),
            "mean_px": float((w * PX).sum()) / s if s else 0.0,
            "mean_py": float((w * PY).sum()) / s if s else 0.0,
            "energy": cell * float((w * e).sum())}

"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the test oracle and by the GPU path, so it holds no
arithmetic of the method itself (no push, no deposit, no mass-matrix solve):
only lattice geometry, initial densities evaluated at lattice nodes, and the
random draws that choose instance parameters.

Lattice convention (the paper only says coordinates are periodic and momenta
open, Sec. "Numerical Examples"): a periodic axis of ``n`` nodes spans
``[lo, hi)`` with ``h = (hi - lo) / n``; an open axis has nodes at both ends,
``h = (hi - lo) / (n - 1)``.  Arrays are ``[n_p][n_x]`` with x fastest.
Initial weights are nodal values of ``f0`` (tent functions interpolate).

Random numbers come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Hamiltonian kinds, numbered as in the C interface (include/vp.h).
H_FREE, H_SHO_EXACT, H_PENDULUM, H_FEL = 0, 1, 2, 3
FEL_DKD, FEL_RK4 = 0, 1   # FEL integrators


@dataclass(frozen=True)
class Axis:
    lo: float
    hi: float
    n: int
    periodic: bool

    @property
    def h(self) -> float:
        return (self.hi - self.lo) / (self.n if self.periodic else self.n - 1)

    def nodes(self) -> np.ndarray:
        return self.lo + np.arange(self.n, dtype=np.float64) * self.h


@dataclass(frozen=True)
class Hamiltonian:
    kind: int
    a: float = 0.0           # pendulum: V(x) = -a cos x
    omega: float = 1.0       # exact rotation: angle per unit time
    fel_delta: float = 0.0   # FEL detuning
    fel_sigma2: float = 0.0  # FEL space-charge coefficient
    A_re: float = 0.0        # FEL field at the current step
    A_im: float = 0.0
    integrator: int = 0      # FEL: FEL_DKD (exact-kick drift-kick-drift) or FEL_RK4


@dataclass
class Instance:
    """One solve: lattice, Hamiltonian, initial weights, time step, step count."""
    name: str
    x: Axis
    p: Axis
    ham: Hamiltonian
    w0: np.ndarray           # float64 [n_p][n_x]
    dt: float
    steps: int
    meta: dict = field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return self.x.n * self.p.n


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def pendulum_axes(nx: int, npp: int | None = None) -> tuple[Axis, Axis]:
    npp = nx if npp is None else npp
    return Axis(-math.pi, math.pi, nx, True), Axis(-3.0, 3.0, npp, False)


def fel_axes(nx: int, npp: int | None = None) -> tuple[Axis, Axis]:
    npp = nx if npp is None else npp
    return Axis(0.0, 2.0 * math.pi, nx, True), Axis(-0.5, 0.5, npp, False)


def _wrapped(d: np.ndarray, period: float) -> np.ndarray:
    """Minimal-image distance on a periodic axis."""
    return (d + 0.5 * period) % period - 0.5 * period


def gaussian(x: Axis, p: Axis, xc: float, pc: float, sigma: float) -> np.ndarray:
    gx = np.exp(-_wrapped(x.nodes() - xc, x.hi - x.lo) ** 2 / (2 * sigma**2)) if x.periodic \
        else np.exp(-(x.nodes() - xc) ** 2 / (2 * sigma**2))
    gp = np.exp(-(p.nodes() - pc) ** 2 / (2 * sigma**2))
    return np.outer(gp, gx)


# --- the five workloads -------------------------------------------------------

def pendulum_gaussian(n: int = 128, seed: int = 1, steps: int = 200) -> Instance:
    """128^2 pendulum, Gaussian at (0, 1), sigma 0.3, plus a U[0,1) 1e-3 floor; dt 0.05."""
    x, p = pendulum_axes(n)
    w0 = gaussian(x, p, 0.0, 1.0, 0.3) + 1e-3 * rng(seed).random((n, n))
    return Instance("pendulum_gaussian", x, p, Hamiltonian(H_PENDULUM, a=1.0), w0, 0.05, steps,
                    {"seed": seed})


def pendulum_band(n: int = 2048, seed: int = 2, steps: int = 1000) -> Instance:
    """Uniform band |p| <= 2.5 straddling the separatrix, 1% multiplicative noise; dt 0.02."""
    x, p = pendulum_axes(n)
    band = (np.abs(p.nodes()) <= 2.5).astype(np.float64)[:, None]
    w0 = band * (1.0 + 0.01 * rng(seed).uniform(-1.0, 1.0, (n, n)))
    return Instance("pendulum_band", x, p, Hamiltonian(H_PENDULUM, a=1.0), w0, 0.02, steps,
                    {"seed": seed})


def fel_gaussian(n: int = 1024, steps: int = 2000, npp: int | None = None) -> Instance:
    """1-D FEL: Gaussian in eta (sigma 0.05) times (1 + 0.01 cos psi); A0 = 1e-3; dz 0.01."""
    x, p = fel_axes(n, npp)
    w0 = np.outer(np.exp(-p.nodes() ** 2 / (2 * 0.05**2)), 1.0 + 0.01 * np.cos(x.nodes()))
    return Instance("fel_gaussian", x, p, Hamiltonian(H_FEL, A_re=1e-3), w0, 0.01, steps)


def fel_flattop(n: int = 256, steps: int = 200, half_width: float = 0.1) -> Instance:
    """FEL start with a hard edge in energy: uniform for |eta| <= 0.1, times (1 + 0.01 cos psi)."""
    x, p = fel_axes(n)
    w0 = np.outer((np.abs(p.nodes()) <= half_width).astype(np.float64),
                  1.0 + 0.01 * np.cos(x.nodes()))
    return Instance("fel_flattop", x, p, Hamiltonian(H_FEL, A_re=1e-3), w0, 0.01, steps)


def _pendulum_request(g: np.random.Generator, n: int, steps: int, dt: float = 0.05) -> Instance:
    x, p = pendulum_axes(n)
    a = g.uniform(0.5, 2.0)
    xc = g.uniform(-math.pi, math.pi)
    pc = g.uniform(-1.5, 1.5)
    return Instance("pendulum_gaussian", x, p, Hamiltonian(H_PENDULUM, a=a),
                    gaussian(x, p, xc, pc, 0.3), dt, steps, {"xc": xc, "pc": pc})


def batch_instances(count: int = 256, seed: int = 4, steps: int = 500,
                    n_min: int = 64, n_max: int = 1024) -> list[Instance]:
    """Uneven pendulum instances: n log-uniform in [n_min, n_max], a ~ U[0.5, 2],
    Gaussian (sigma 0.3) with centre x ~ U[-pi, pi), p ~ U[-1.5, 1.5]; dt 0.05."""
    g = rng(seed)
    out = []
    for _ in range(count):
        n = int(round(math.exp(g.uniform(math.log(n_min), math.log(n_max)))))
        out.append(_pendulum_request(g, n, steps))
    return out


@dataclass
class Request:
    rid: int
    arrival: float           # seconds after the start of the trace
    kind: int                # H_PENDULUM or H_FEL
    n: int
    steps: int
    seed: int                # per-request seed for its own initial condition draws

    def instance(self) -> Instance:
        if self.kind == H_FEL:
            inst = fel_gaussian(self.n, self.steps)
        else:
            inst = _pendulum_request(rng(self.seed), self.n, self.steps)
        inst.meta["rid"] = self.rid
        return inst


def request_trace(count: int = 1000, seed: int = 5, rate: float = 100.0,
                  n_min: int = 128, n_max: int = 2048, steps_min: int = 100,
                  steps_max: int = 2000, fel_fraction: float = 0.3) -> list[Request]:
    """Poisson arrivals (rate per second) of mixed pendulum / FEL requests."""
    g = rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += g.exponential(1.0 / rate)
        kind = H_FEL if g.random() < fel_fraction else H_PENDULUM
        n = int(round(math.exp(g.uniform(math.log(n_min), math.log(n_max)))))
        steps = int(g.integers(steps_min, steps_max + 1))
        out.append(Request(rid, t, kind, n, steps, int(g.integers(0, 2**31 - 1))))
    return out


# --- the 2D2V phase space (x, y, p_x, p_y) -----------------------------------

def phase4d_axes(n: int, npp: int, pmax: float = 3.0) -> tuple[Axis, Axis, Axis, Axis]:
    """x, y periodic on [-pi, pi) with n nodes; p_x, p_y open on [-pmax, pmax] with npp nodes."""
    return (Axis(-math.pi, math.pi, n, True), Axis(-math.pi, math.pi, n, True),
            Axis(-pmax, pmax, npp, False), Axis(-pmax, pmax, npp, False))


def phase4d_thermal(axes, seed: int = 7, sigma: float = 0.8) -> np.ndarray:
    """A state near equilibrium in V = -cos x - cos y: exp(-|p|^2 / (2 sigma^2))
    exp(cos x + cos y) at the nodes, times seeded U[0.9, 1.1] noise per node.
    float64 [n_py][n_px][n_y][n_x]."""
    x, y, px, py = axes
    g = rng(seed)
    shape = (py.n, px.n, y.n, x.n)
    w = (np.exp(-(py.nodes()[:, None, None, None] ** 2 + px.nodes()[None, :, None, None] ** 2) / (2 * sigma**2))
         * np.exp(np.cos(y.nodes())[None, None, :, None] + np.cos(x.nodes())[None, None, None, :]))
    return w * g.uniform(0.9, 1.1, shape)

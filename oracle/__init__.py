"""FP64 CPU oracle of the phase-space-conservation Vlasov step (test infrastructure).

Only the tests, the GPU smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library never does.  The numerics live in
``vp_oracle.c`` (plain C, FP64); ``brute.py`` holds quadrature and dense
linear-algebra checks for tiny grids; ``spline_basis.py`` is the method with
quadratic or cubic B-spline basis functions.  See ``vp_oracle.c`` for the equations
followed and the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vp_oracle.c")
_LIB = os.path.join(_HERE, "libvp_oracle.so")

# portable flags: the built library is also run on other hosts
CFLAGS = ["-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall"]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Axis(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("n", C.c_int32), ("periodic", C.c_int32)]


class _Ham(C.Structure):
    _fields_ = [("kind", C.c_int32), ("integrator", C.c_int32), ("a", C.c_double),
                ("omega", C.c_double), ("fel_delta", C.c_double), ("fel_sigma2", C.c_double)]


MOMENT_FIELDS = ("sum_w", "mass", "neg_mass", "l1", "entropy", "mean_p", "energy",
                 "A_re", "A_im", "bunch_re", "bunch_im", "fel_invariant")


class _Moments(C.Structure):
    _fields_ = [(f, C.c_double) for f in MOMENT_FIELDS] + [("step", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        P = C.POINTER
        dp = P(C.c_double)
        L.orc_b3.restype = C.c_double
        L.orc_b3.argtypes = [C.c_double]
        L.orc_push.argtypes = [P(_Axis), P(_Axis), P(_Ham), C.c_double, dp, dp, dp]
        L.orc_deposit.argtypes = [P(_Axis), P(_Axis), dp, dp, dp, dp]
        L.orc_solve.argtypes = [P(_Axis), P(_Axis), dp]
        L.orc_bunching.argtypes = [P(_Axis), P(_Axis), P(_Ham), C.c_double, dp, C.c_double, dp]
        L.orc_push_rk4.argtypes = [P(_Axis), P(_Axis), P(_Ham), C.c_double, dp, C.c_double, dp, dp, dp, dp]
        L.orc_moments_of.argtypes = [P(_Axis), P(_Axis), P(_Ham), dp, dp, C.c_double, C.c_int64,
                                     P(_Moments)]
        L.orc_run.argtypes = [P(_Axis), P(_Axis), P(_Ham), C.c_double, C.c_int64, dp, dp,
                              C.c_double, C.c_int32, P(_Moments)]
        L.orc_run.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _ax(a) -> _Axis:
    return _Axis(float(a.lo), float(a.hi), int(a.n), int(bool(a.periodic)))


def _ham(h) -> _Ham:
    return _Ham(int(h.kind), int(getattr(h, "integrator", 0)), float(h.a), float(h.omega),
                float(h.fel_delta), float(h.fel_sigma2))


def _dptr(arr: np.ndarray):
    assert arr.dtype == np.float64 and arr.flags.c_contiguous
    return arr.ctypes.data_as(C.POINTER(C.c_double))


def b3(s: float) -> float:
    return lib().orc_b3(float(s))


def push(x, p, ham, dt, At=None):
    """Per-node displacement in cell units: (du, dv), each [n_p][n_x]."""
    du = np.empty((p.n, x.n))
    dv = np.empty((p.n, x.n))
    at = None if At is None else np.ascontiguousarray(At, dtype=np.float64)
    lib().orc_push(_ax(x), _ax(p), _ham(ham), float(dt), None if at is None else _dptr(at),
                   _dptr(du), _dptr(dv))
    return du, dv


def deposit(x, p, du, dv, w):
    """b = Delta^T w without the h_x h_p factor."""
    du, dv, w = (np.ascontiguousarray(a, dtype=np.float64) for a in (du, dv, w))
    b = np.empty((p.n, x.n))
    lib().orc_deposit(_ax(x), _ax(p), _dptr(du), _dptr(dv), _dptr(w), _dptr(b))
    return b


def solve(x, p, b):
    """(M_x^{-1} (x) M_p^{-1}) b."""
    out = np.array(b, dtype=np.float64, order="C", copy=True)
    lib().orc_solve(_ax(x), _ax(p), _dptr(out))
    return out


def push_rk4(x, p, ham, dz, w, N0, A):
    """One FEL Runge-Kutta step of every node: displacements (du, dv) in cells
    and the new field."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    a = np.array([complex(A).real, complex(A).imag])
    du = np.empty((p.n, x.n))
    dv = np.empty((p.n, x.n))
    an = np.zeros(2)
    lib().orc_push_rk4(_ax(x), _ax(p), _ham(ham), float(dz), _dptr(w), float(N0), _dptr(a), _dptr(du),
                       _dptr(dv), _dptr(an))
    return du, dv, complex(an[0], an[1])


def bunching(x, p, ham, dz, w, N0):
    out = np.zeros(2)
    w = np.ascontiguousarray(w, dtype=np.float64)
    lib().orc_bunching(_ax(x), _ax(p), _ham(ham), float(dz), _dptr(w), float(N0), _dptr(out))
    return complex(out[0], out[1])


def _moments_dict(m: _Moments) -> dict:
    d = {f: getattr(m, f) for f in MOMENT_FIELDS}
    d["step"] = m.step
    return d


def moments(x, p, ham, w, A=0j, N0=None, step=0) -> dict:
    w = np.ascontiguousarray(w, dtype=np.float64)
    N0 = float(w.sum()) if N0 is None else float(N0)
    a = np.array([complex(A).real, complex(A).imag])
    m = _Moments()
    lib().orc_moments_of(_ax(x), _ax(p), _ham(ham), _dptr(w), _dptr(a), N0, int(step), C.byref(m))
    return _moments_dict(m)


@dataclass
class RunResult:
    w: np.ndarray
    A: complex
    series: list | None


def run(x, p, ham, w0, dt, steps, A0=None, N0=None, round_fp32=False, series=False) -> RunResult:
    """Advance ``w0`` by ``steps`` steps.  For the FEL, A0 defaults to the
    Hamiltonian's field and N0 to sum(w0)."""
    w = np.array(w0, dtype=np.float64, order="C", copy=True)
    if A0 is None:
        A0 = complex(getattr(ham, "A_re", 0.0), getattr(ham, "A_im", 0.0))
    a = np.array([complex(A0).real, complex(A0).imag])
    N0 = float(w.sum()) if N0 is None else float(N0)
    ser = (_Moments * max(int(steps), 1))() if series else None
    rc = lib().orc_run(_ax(x), _ax(p), _ham(ham), float(dt), int(steps), _dptr(w), _dptr(a), N0,
                       int(bool(round_fp32)), ser)
    if rc != 0:
        raise RuntimeError(f"orc_run failed with {rc}")
    out = [_moments_dict(ser[i]) for i in range(int(steps))] if series else None
    return RunResult(w, complex(a[0], a[1]), out)


def run_instance(inst, steps=None, **kw) -> RunResult:
    return run(inst.x, inst.p, inst.ham, inst.w0, inst.dt, inst.steps if steps is None else steps,
               **kw)


def threads() -> int:
    return int(lib().orc_max_threads())


def rel_l1(a: np.ndarray, ref: np.ndarray) -> float:
    """||a - ref||_1 / ||ref||_1."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(a - ref).sum() / np.abs(ref).sum())


if __name__ == "__main__":  # pragma: no cover
    print(build(force="--force" in sys.argv))

"""ctypes binding of libvp (include/vp.h): argument marshalling only.

Every step of the method runs in the HIP kernels of ``libvp.so``; this module
moves pointers and sizes across the C interface and turns status codes into
exceptions.  PyTorch provides device memory (the grid workspace) and streams.
If the library has not been built, ``lib()`` raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vp.h")

VP_OK, VP_EINVAL, VP_ENOMEM, VP_ESTATE, VP_EHIP, VP_EUNSUPPORTED, VP_ENONFINITE, VP_ERANGE = 0, -1, -2, -3, -4, -5, -6, -7
H_FREE, H_SHO_EXACT, H_PENDULUM, H_FEL = 0, 1, 2, 3
BASIS_TENT, BASIS_QUADRATIC, BASIS_CUBIC = 0, 1, 2


class VpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vp error {code}: {msg}")
        self.code = code


class Axis(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("n", C.c_int32), ("periodic", C.c_int32)]


class GridDesc(C.Structure):
    _fields_ = [("x", Axis), ("p", Axis), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("stream", C.c_void_p)]


class Hamiltonian(C.Structure):
    _fields_ = [("kind", C.c_int32), ("integrator", C.c_int32), ("a", C.c_double), ("omega", C.c_double),
                ("fel_delta", C.c_double), ("fel_sigma2", C.c_double), ("A_re", C.c_double),
                ("A_im", C.c_double)]


MOMENT_FIELDS = ("sum_w", "mass", "neg_mass", "l1", "entropy", "mean_p", "energy", "A_re", "A_im",
                 "bunch_re", "bunch_im", "fel_invariant")


class Moments(C.Structure):
    _fields_ = [(f, C.c_double) for f in MOMENT_FIELDS] + [("step", C.c_int64), ("nonfinite", C.c_int64)]


class Grid4Desc(C.Structure):
    _fields_ = [("axes", Axis * 4), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("stream", C.c_void_p)]


class Hamiltonian4(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a", C.c_double), ("b", C.c_double), ("c", C.c_double)]


MOMENT4_FIELDS = ("sum_w", "mass", "neg_mass", "l1", "entropy", "mean_px", "mean_py", "energy")


class Moments4(C.Structure):
    _fields_ = [(f, C.c_double) for f in MOMENT4_FIELDS] + [("step", C.c_int64), ("nonfinite", C.c_int64)]


class RunState(C.Structure):
    _fields_ = [("fix_exponent", C.c_int32), ("reserved", C.c_int32), ("step", C.c_int64), ("n0", C.c_double),
                ("bunch_dz", C.c_double), ("fel", C.c_double * 16)]


class Tiles(C.Structure):
    _fields_ = [("k1_tx", C.c_int32), ("k1_ty", C.c_int32), ("k1_threads", C.c_int32)]


_lib = None


def declared_functions() -> list[str]:
    """Names of the functions include/vp.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(vp_\w+)\s*\(", text, re.M)))


def lib(load_torch: bool = True):
    """Load libvp.so.  PyTorch is imported first so that the library binds to the
    HIP runtime PyTorch already uses (one runtime per process)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                           "(or python paper_2007_12227_amd/build.py)")
    if load_torch:
        import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    L.vp_workspace_bytes.restype = C.c_size_t
    L.vp_workspace_bytes.argtypes = [P(Axis), P(Axis)]
    L.vp_create_grid.argtypes = [P(GridDesc), P(C.c_void_p)]
    L.vp_destroy_grid.argtypes = [C.c_void_p]
    L.vp_set_hamiltonian.argtypes = [C.c_void_p, P(Hamiltonian)]
    L.vp_set_density.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
    L.vp_get_density.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
    L.vp_step.argtypes = [C.c_void_p, C.c_double, C.c_int64]
    L.vp_moments.argtypes = [C.c_void_p, P(Moments)]
    L.vp_step_timed.argtypes = [C.c_void_p, C.c_double, C.c_int64, P(C.c_double)]
    L.vp_set_tiles.argtypes = [C.c_void_p, P(Tiles)]
    L.vp_get_tiles.argtypes = [C.c_void_p, P(Tiles)]
    L.vp_set_launch.argtypes = [C.c_void_p, C.c_int32]
    L.vp_autotune.argtypes = [C.c_void_p, C.c_double, P(C.c_double)]
    L.vp_batch_create.argtypes = [P(C.c_void_p), C.c_int32, P(C.c_double), P(C.c_void_p)]
    L.vp_batch_step.argtypes = [C.c_void_p, C.c_int64]
    L.vp_batch_step_timed.argtypes = [C.c_void_p, C.c_int64, P(C.c_double)]
    L.vp_batch_destroy.argtypes = [C.c_void_p]
    L.vp_batch_autotune.argtypes = [C.c_void_p, P(C.c_double)]
    L.vp_batch_config.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32), P(C.c_int32)]
    L.vp_status_string.restype = C.c_char_p
    L.vp_status_string.argtypes = [C.c_int]
    L.vp_last_error.restype = C.c_char_p
    L.vp_plan_source_box.argtypes = [P(Axis), P(Axis), P(Hamiltonian), C.c_int32, C.c_double, C.c_double,
                                     C.c_double, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P(C.c_int32)]
    L.vp_set_basis.argtypes = [C.c_void_p, C.c_int32]
    L.vp_set_fixed_point.argtypes = [C.c_void_p, C.c_int32]
    L.vp_set_map_cache.argtypes = [C.c_void_p, C.c_int32]
    L.vp_get_run_state.argtypes = [C.c_void_p, P(RunState)]
    L.vp_set_run_state.argtypes = [C.c_void_p, P(RunState)]
    L.vp_step_noalloc.argtypes = [P(Axis), P(Axis), P(Hamiltonian), C.c_int32, C.c_double, C.c_int64,
                                  C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
    L.vp4_workspace_bytes.restype = C.c_size_t
    L.vp4_workspace_bytes.argtypes = [P(Axis)]
    L.vp4_create_grid.argtypes = [P(Grid4Desc), P(C.c_void_p)]
    L.vp4_destroy_grid.argtypes = [C.c_void_p]
    L.vp4_set_hamiltonian.argtypes = [C.c_void_p, P(Hamiltonian4)]
    L.vp4_set_tiles.argtypes = [C.c_void_p, P(C.c_int32)]
    L.vp4_set_density.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
    L.vp4_get_density.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
    L.vp4_step.argtypes = [C.c_void_p, C.c_double, C.c_int64]
    L.vp4_step_timed.argtypes = [C.c_void_p, C.c_double, C.c_int64, P(C.c_double)]
    L.vp4_autotune.argtypes = [C.c_void_p, C.c_double, P(C.c_double)]
    L.vp4_get_tiles.argtypes = [C.c_void_p, P(C.c_int32)]
    L.vp4_moments.argtypes = [C.c_void_p, P(Moments4)]
    L.vp4_plan_source_box.argtypes = [P(Axis), P(Hamiltonian4), C.c_double, P(C.c_int32), P(C.c_int32),
                                      P(C.c_int32)]
    for name in declared_functions():
        if name not in ("vp_workspace_bytes", "vp4_workspace_bytes", "vp_status_string", "vp_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc: int) -> int:
    if rc != VP_OK:
        raise VpError(rc, lib().vp_last_error().decode())
    return rc


def axis(a) -> Axis:
    return Axis(float(a.lo), float(a.hi), int(a.n), int(bool(a.periodic)))


def hamiltonian(h) -> Hamiltonian:
    return Hamiltonian(int(h.kind), int(getattr(h, "integrator", 0)), float(getattr(h, "a", 0.0)),
                       float(getattr(h, "omega", 1.0)),
                       float(getattr(h, "fel_delta", 0.0)), float(getattr(h, "fel_sigma2", 0.0)),
                       float(getattr(h, "A_re", 0.0)), float(getattr(h, "A_im", 0.0)))


def workspace_bytes(x, p) -> int:
    return int(lib().vp_workspace_bytes(C.byref(axis(x)), C.byref(axis(p))))


def plan_source_box(x, p, ham, dt, kick=0j, bx=(0, 0), by=(0, 0), basis=BASIS_TENT) -> tuple[int, int, int, int]:
    box = (C.c_int32 * 4)()
    check(lib().vp_plan_source_box(C.byref(axis(x)), C.byref(axis(p)), C.byref(hamiltonian(ham)), int(basis),
                                   float(dt), float(complex(kick).real), float(complex(kick).imag),
                                   int(bx[0]), int(bx[1]), int(by[0]), int(by[1]), box))
    return tuple(int(v) for v in box)


def plan_source_box4(axes, kind, a, b, c, dt, tile_lo, tile_hi) -> tuple:
    """The 2D2V deposit's source box of a tile (vp4_plan_source_box): ((lo, hi) per axis x, y, p_x, p_y)."""
    ax = (Axis * 4)(*[axis(v) for v in axes])
    box = (C.c_int32 * 8)()
    check(lib().vp4_plan_source_box(ax, C.byref(Hamiltonian4(int(kind), float(a), float(b), float(c))), float(dt),
                                    (C.c_int32 * 4)(*[int(v) for v in tile_lo]),
                                    (C.c_int32 * 4)(*[int(v) for v in tile_hi]), box))
    return tuple((int(box[2 * d]), int(box[2 * d + 1])) for d in range(4))


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Grid:
    """One lattice with its device state; all work runs on ``stream``."""

    def __init__(self, x, p, stream=None, device="cuda"):
        import torch
        self.x, self.p = x, p
        nbytes = workspace_bytes(x, p)
        if nbytes == 0:
            check(VP_EINVAL)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        self._ws_ptr = base + (-base) % 256
        self.stream = stream
        desc = GridDesc(axis(x), axis(p), C.c_void_p(self._ws_ptr), nbytes, _stream_handle(stream))
        h = C.c_void_p()
        check(lib().vp_create_grid(C.byref(desc), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().vp_destroy_grid(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_hamiltonian(self, ham):
        check(lib().vp_set_hamiltonian(self._h, C.byref(hamiltonian(ham))))

    def set_basis(self, basis: int):
        """BASIS_TENT, BASIS_QUADRATIC or BASIS_CUBIC (B-spline basis functions)."""
        check(lib().vp_set_basis(self._h, int(basis)))

    def set_density(self, w):
        import torch
        if isinstance(w, torch.Tensor) and w.is_cuda:
            t = w.to(torch.float32).contiguous()
            assert t.numel() == self.x.n * self.p.n
            check(lib().vp_set_density(self._h, C.c_void_p(t.data_ptr()), 1))
        else:
            a = np.ascontiguousarray(w, dtype=np.float32)
            assert a.size == self.x.n * self.p.n
            check(lib().vp_set_density(self._h, a.ctypes.data_as(C.c_void_p), 0))

    def density(self) -> np.ndarray:
        out = np.empty((self.p.n, self.x.n), dtype=np.float32)
        check(lib().vp_get_density(self._h, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def density_into(self, t):
        """Copy the state into a CUDA float32 tensor of n_p*n_x elements."""
        check(lib().vp_get_density(self._h, C.c_void_p(t.data_ptr()), 1))
        return t

    def step(self, dt: float, n: int = 1):
        check(lib().vp_step(self._h, float(dt), int(n)))

    def step_timed(self, dt: float, n: int) -> tuple[float, float]:
        """n steps with per-kernel HIP events: mean (deposit, solve) microseconds."""
        us = (C.c_double * 2)()
        check(lib().vp_step_timed(self._h, float(dt), int(n), us))
        return us[0], us[1]

    def moments(self, check_state: bool = True) -> dict:
        """FP64 diagnostics.  A state with NaN/Inf weights or a deposit that
        left its fixed-point range raises VpError (VP_ENONFINITE, VP_ERANGE);
        with check_state=False the moments are returned anyway, with the code
        in d["status"]."""
        m = Moments()
        rc = lib().vp_moments(self._h, C.byref(m))
        d = {f: getattr(m, f) for f in MOMENT_FIELDS}
        d["step"], d["nonfinite"] = m.step, m.nonfinite
        if check_state or rc not in (VP_OK, VP_ENONFINITE, VP_ERANGE):
            check(rc)
        d["status"] = rc
        return d

    def run_state(self) -> RunState:
        """The scalars of the run beside the weights (vp_get_run_state)."""
        st = RunState()
        check(lib().vp_get_run_state(self._h, C.byref(st)))
        return st

    def set_run_state(self, st: RunState):
        check(lib().vp_set_run_state(self._h, C.byref(st)))

    def set_fixed_point(self, e: int):
        """Exponent of the deposit's fixed-point cell sums (vp_set_fixed_point)."""
        check(lib().vp_set_fixed_point(self._h, int(e)))

    def set_tiles(self, k1=(0, 0), threads: int = 0):
        """Deposit launch shape: tile (columns, rows) and threads per workgroup
        (zero keeps the current value)."""
        check(lib().vp_set_tiles(self._h, C.byref(Tiles(k1[0], k1[1], threads))))

    def tiles(self) -> dict:
        t = Tiles()
        check(lib().vp_get_tiles(self._h, C.byref(t)))
        return {"k1": (t.k1_tx, t.k1_ty), "threads": t.k1_threads}

    def set_map_cache(self, on: bool):
        """Cache the push of a static Hamiltonian (vp_set_map_cache)."""
        check(lib().vp_set_map_cache(self._h, int(bool(on))))

    def set_launch(self, use_graph: bool):
        check(lib().vp_set_launch(self._h, int(bool(use_graph))))

    def autotune(self, dt: float, cached: bool = False) -> float:
        """Pick tile shapes by timing candidates; with cached=True reuse the
        choice made for the same shape class if there is one (returns 0.0)."""
        if cached:
            check(lib().vp_autotune(self._h, float(dt), None))
            return 0.0
        us = C.c_double()
        check(lib().vp_autotune(self._h, float(dt), C.byref(us)))
        return us.value


class Batch:
    """Grids advanced together: one launch per kernel covers every tile of every grid."""

    def __init__(self, grids: list[Grid], dts: list[float]):
        self.grids = list(grids)
        arr = (C.c_void_p * len(grids))(*[g.handle.value for g in grids])
        d = (C.c_double * len(grids))(*[float(v) for v in dts])
        h = C.c_void_p()
        check(lib().vp_batch_create(arr, len(grids), d, C.byref(h)))
        self._h = h

    def step(self, n: int = 1):
        check(lib().vp_batch_step(self._h, int(n)))

    def step_timed(self, n: int) -> tuple[float, float]:
        """n batch steps with per-kernel HIP events: mean (deposit, solve) microseconds."""
        us = (C.c_double * 2)()
        check(lib().vp_batch_step_timed(self._h, int(n), us))
        return us[0], us[1]

    def autotune(self, cached: bool = False) -> float:
        """Pick the batch's launch configuration by timing (vp_batch_autotune);
        cached=True applies a choice made for the same composition class."""
        if cached:
            check(lib().vp_batch_autotune(self._h, None))
            return 0.0
        us = C.c_double()
        check(lib().vp_batch_autotune(self._h, C.byref(us)))
        return us.value

    def config(self) -> dict:
        g, t, n = C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().vp_batch_config(self._h, C.byref(g), C.byref(t), C.byref(n)))
        return {"deposit_grid": g.value, "deposit_threads": t.value, "deposit_tiles": n.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().vp_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_noalloc(x, p, ham, dt, nsteps, w_in, w_out, basis=BASIS_TENT, fel_n0=0.0, fel_A=None, status=None,
                 stream=None):
    """vp_step_noalloc on CUDA tensors: w_in, w_out float32 [n_p][n_x]; fel_A a
    float64 tensor of 2 (FEL); status an int32 tensor of 1 (optional)."""
    import torch
    for t in (w_in, w_out):
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == x.n * p.n
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
    check(lib().vp_step_noalloc(C.byref(axis(x)), C.byref(axis(p)), C.byref(hamiltonian(ham)), int(basis),
                                float(dt), int(nsteps), ptr(w_in), ptr(w_out), float(fel_n0), ptr(fel_A),
                                ptr(status), _stream_handle(stream)))


def workspace_bytes4(axes) -> int:
    arr = (Axis * 4)(*[axis(a) for a in axes])
    return int(lib().vp4_workspace_bytes(arr))


class Grid4:
    """A four-dimensional (x, y, p_x, p_y) lattice; weights [n_py][n_px][n_y][n_x]."""

    def __init__(self, axes, stream=None, device="cuda"):
        import torch
        self.axes = tuple(axes)
        self.shape = tuple(a.n for a in reversed(self.axes))
        nbytes = workspace_bytes4(self.axes)
        if nbytes == 0:
            check(VP_EINVAL)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        ptr = base + (-base) % 256
        desc = Grid4Desc((Axis * 4)(*[axis(a) for a in self.axes]), C.c_void_p(ptr), nbytes, _stream_handle(stream))
        h = C.c_void_p()
        check(lib().vp4_create_grid(C.byref(desc), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().vp4_destroy_grid(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_hamiltonian(self, kind: int, a: float = 0.0, b: float = 0.0, c: float = 0.0):
        check(lib().vp4_set_hamiltonian(self._h, C.byref(Hamiltonian4(int(kind), float(a), float(b), float(c)))))

    def set_tiles(self, tile):
        check(lib().vp4_set_tiles(self._h, (C.c_int32 * 4)(*[int(v) for v in tile])))

    def tiles(self) -> tuple:
        t = (C.c_int32 * 4)()
        check(lib().vp4_get_tiles(self._h, t))
        return tuple(t)

    def autotune(self, dt: float, cached: bool = False) -> float:
        """Pick the deposit tile by timing (vp4_autotune); cached=True applies
        the choice made for the same shape class (returns 0.0)."""
        if cached:
            check(lib().vp4_autotune(self._h, float(dt), None))
            return 0.0
        us = C.c_double()
        check(lib().vp4_autotune(self._h, float(dt), C.byref(us)))
        return us.value

    def set_density(self, w):
        a = np.ascontiguousarray(w, dtype=np.float32)
        assert a.shape == self.shape, (a.shape, self.shape)
        check(lib().vp4_set_density(self._h, a.ctypes.data_as(C.c_void_p), 0))

    def density(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float32)
        check(lib().vp4_get_density(self._h, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def step(self, dt: float, n: int = 1):
        check(lib().vp4_step(self._h, float(dt), int(n)))

    def step_timed(self, dt: float, n: int) -> tuple[float, float]:
        us = (C.c_double * 2)()
        check(lib().vp4_step_timed(self._h, float(dt), int(n), us))
        return us[0], us[1]

    def moments(self) -> dict:
        m = Moments4()
        check(lib().vp4_moments(self._h, C.byref(m)))
        d = {f: getattr(m, f) for f in MOMENT4_FIELDS}
        d["step"], d["nonfinite"] = m.step, m.nonfinite
        return d


def grid_for(inst, stream=None) -> Grid:
    """A grid holding an input instance (paper_2007_12227_amd.inputs.Instance)."""
    g = Grid(inst.x, inst.p, stream)
    g.set_hamiltonian(inst.ham)
    g.set_density(inst.w0)
    return g

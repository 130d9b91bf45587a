"""Host-side tests of the C interface: symbols, validation, planning.  No GPU."""
import ctypes as C
import math

import numpy as np
import pytest

import oracle
from paper_2007_12227_amd import binding as B
from paper_2007_12227_amd.inputs import (H_FEL, H_FREE, H_PENDULUM, H_SHO_EXACT, Axis, Hamiltonian,
                                         fel_axes, pendulum_axes, rng)


@pytest.fixture(scope="module")
def L():
    return B.lib()


def test_library_exports_every_declared_symbol(L):
    names = B.declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name


def test_workspace_bytes(L):
    x, p = pendulum_axes(128)
    n1 = B.workspace_bytes(x, p)
    assert n1 >= 3 * 128 * 128 * 4
    assert B.workspace_bytes(*pendulum_axes(256)) > n1
    assert L.vp_workspace_bytes(C.byref(B.Axis(0, 1, 3, 1)), C.byref(B.axis(p))) == 0
    assert L.vp_workspace_bytes(C.byref(B.Axis(1, 0, 16, 1)), C.byref(B.axis(p))) == 0
    assert L.vp_workspace_bytes(None, C.byref(B.axis(p))) == 0


def _create(L, x, p, ws, nbytes):
    desc = B.GridDesc(x, p, C.c_void_p(ws), nbytes, None)
    h = C.c_void_p()
    return L.vp_create_grid(C.byref(desc), C.byref(h)), h


def test_create_grid_validation(L):
    x, p = pendulum_axes(64)
    need = B.workspace_bytes(x, p)
    assert L.vp_create_grid(None, None) == B.VP_EINVAL
    assert _create(L, B.Axis(0, 1, 2, 1), B.axis(p), 256, need)[0] == B.VP_EINVAL
    assert _create(L, B.axis(x), B.Axis(-1, 1, 64, 1), 256, need)[0] == B.VP_EUNSUPPORTED
    assert _create(L, B.axis(x), B.axis(p), 0, need)[0] == B.VP_ENOMEM
    assert _create(L, B.axis(x), B.axis(p), 256, need - 1)[0] == B.VP_ENOMEM
    assert _create(L, B.axis(x), B.axis(p), 258, need)[0] == B.VP_EINVAL
    assert b"256-byte" in L.vp_last_error()


def test_null_handles(L):
    assert L.vp_destroy_grid(None) == B.VP_OK
    assert L.vp_batch_destroy(None) == B.VP_OK
    assert L.vp_step(None, 0.1, 1) == B.VP_EINVAL
    assert L.vp_moments(None, None) == B.VP_EINVAL
    assert L.vp_set_hamiltonian(None, None) == B.VP_EINVAL
    assert L.vp_batch_step(None, 1) == B.VP_EINVAL
    assert L.vp_set_basis(None, B.BASIS_CUBIC) == B.VP_EINVAL
    assert L.vp_set_fixed_point(None, 0) == B.VP_EINVAL
    assert L.vp_batch_create(None, 0, None, None) == B.VP_EINVAL


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.vp_status_string(code)
    assert L.vp_status_string(-99) == b"unknown status"


# ---- the deposit tile's source box: every node that reaches the tile is in it ----

def _check_box(x, p, ham, dt, kick, tile, box, wide=0):
    """A moved tent at cell position u touches columns floor(u)-1 .. floor(u)+2;
    a B-spline basis function of degree wide + 1, floor(u)-1-wide .. floor(u)+2+wide.
    The FP64 push of the oracle is also moved by +-1e-4 cells (the FP32 push's
    rounding is ~1e-6 cells)."""
    du, dv = oracle.push(x, p, ham, dt, None if kick is None else np.array([kick.real, kick.imag]))
    bx0, bx1, by0, by1 = tile
    x0, x1, y0, y1 = box
    j, i = np.meshgrid(np.arange(p.n), np.arange(x.n), indexing="ij")
    for delta in (-1e-4, 0.0, 1e-4):
        u = i + du + delta
        v = j + dv + delta
        ku, kv = np.floor(u), np.floor(v)
        row_hit = (kv >= by0 - 2 - wide) & (kv <= by1 + wide)
        shifts = range(-3, 4) if x.periodic else (0,)
        for m in shifts:
            col_hit = (ku + m * x.n >= bx0 - 2 - wide) & (ku + m * x.n <= bx1 + wide)
            hit = row_hit & col_hit
            ii = i[hit] + m * x.n
            jj = j[hit]
            assert np.all((ii >= x0) & (ii < x1)), (tile, box, ii.min(), ii.max())
            assert np.all((jj >= y0) & (jj < y1)), (tile, box, jj.min(), jj.max())


@pytest.mark.parametrize("basis", [B.BASIS_TENT, B.BASIS_QUADRATIC, B.BASIS_CUBIC])
@pytest.mark.parametrize("seed", range(6))
def test_source_box_contains_every_reaching_node(seed, basis):
    g = rng(100 + seed)
    for _ in range(12):
        kind = [H_FREE, H_PENDULUM, H_FEL, H_SHO_EXACT][g.integers(0, 4)]
        n = int(g.integers(16, 160))
        kick = None
        if kind == H_SHO_EXACT:
            half = 3.0
            x = Axis(-half, half, n, False)
            p = Axis(-half, half, int(g.integers(16, 160)), False)
            ham = Hamiltonian(kind, omega=1.0)
            dt = g.uniform(-math.pi, math.pi)
        elif kind == H_FEL:
            x, p = fel_axes(n, int(g.integers(16, 160)))
            ham = Hamiltonian(kind)
            dt = g.uniform(0.005, 0.05)
            kick = complex(*g.uniform(-0.6, 0.6, 2))
        else:
            x, p = pendulum_axes(n, int(g.integers(16, 160)))
            ham = Hamiltonian(kind, a=g.uniform(0.3, 2.5))
            dt = g.uniform(0.005, 0.2)
        tx = int(g.integers(8, max(9, x.n)))
        ty = int(g.integers(1, max(2, p.n // 2)))
        bx0 = int(g.integers(0, x.n)) // tx * tx
        by0 = int(g.integers(0, p.n)) // ty * ty
        tile = (bx0, min(bx0 + tx, x.n), by0, min(by0 + ty, p.n))
        box = B.plan_source_box(x, p, ham, dt, kick if kick is not None else 0j, tile[:2], tile[2:], basis)
        _check_box(x, p, ham, dt, kick, tile, box, wide=basis)


def test_source_box_is_tight_for_smooth_pendulum():
    """The box is the tile shifted by the local displacement, not widened by the
    global maximum: for the 2048^2 pendulum at dt 0.02 a 128x32 tile scans
    under 1.6x its own area."""
    x, p = pendulum_axes(2048)
    ham = Hamiltonian(H_PENDULUM, a=1.0)
    worst = 0.0
    for by0 in range(0, 2048, 32 * 9):
        for bx0 in range(0, 2048, 128 * 3):
            x0, x1, y0, y1 = B.plan_source_box(x, p, ham, 0.02, 0j, (bx0, bx0 + 128), (by0, by0 + 32))
            worst = max(worst, (x1 - x0) * (y1 - y0) / (128 * 32))
    assert worst < 1.6


# ---- the 2D2V deposit tile's source box (vp4_plan_source_box) ----

def _reaches(cells, lo, hi, n, periodic):
    """A moved tent whose pushed cell is `cells` has taps at cells - 1 .. cells + 2:
    does any of them fall in [lo, hi) (modulo n on a periodic axis)?"""
    hit = np.zeros(cells.shape, dtype=bool)
    for m in range(-1, 3):
        c = cells + m
        hit |= ((c % n >= lo) & (c % n < hi)) if periodic else ((c >= lo) & (c < hi))
    return hit


@pytest.mark.parametrize("seed", range(6))
def test_source_box4_contains_every_reaching_node(seed):
    """Every node whose moved 4-D tent deposits into the tile (on all four axes
    at once) lies in the planned box, for the FP64 push of the 2D2V oracle moved
    by +-1e-4 cells (the FP32 push's rounding is ~1e-6)."""
    from oracle import phase4d as P4
    g = rng(300 + seed)
    for _ in range(8):
        n = [int(v) for v in g.integers(6, 20, 4)]
        pm = float(g.uniform(1.0, 4.0))
        axes = (Axis(-math.pi, math.pi, n[0], True), Axis(-math.pi, math.pi, n[1], True),
                Axis(-pm, pm, n[2], False), Axis(-pm, pm, n[3], False))
        kind = [H_FREE, H_PENDULUM][int(g.integers(0, 2))]
        a, b, c = (float(v) for v in g.uniform(-1.5, 1.5, 3))
        dt = float(g.uniform(0.01, 0.6)) if g.random() < 0.8 else float(g.uniform(1.0, 4.0))
        lo = [int(g.integers(0, n[d])) for d in range(4)]
        hi = [int(g.integers(lo[d] + 1, n[d] + 1)) for d in range(4)]
        box = B.plan_source_box4(axes, kind, a, b, c, dt, lo, hi)
        disp = P4.push(axes, P4.Ham4(P4.H4_FREE if kind == H_FREE else P4.H4_POTENTIAL, a, b, c), dt)
        idx = np.meshgrid(*[np.arange(m) for m in reversed(n)], indexing="ij")[::-1]  # x, y, px, py index arrays
        inbox = np.ones(disp[0].shape, dtype=bool)
        for d in range(4):
            bl, bh = box[d]
            assert 0 <= bh - bl <= n[d]
            if d < 2:
                assert 0 <= bl < n[d] or bh == bl
                inbox &= (idx[d] - bl) % n[d] < bh - bl
            else:
                inbox &= (idx[d] >= bl) & (idx[d] < bh)
        for delta in (-1e-4, 0.0, 1e-4):
            reach = np.ones(disp[0].shape, dtype=bool)
            for d in range(4):
                cells = np.floor(idx[d] + disp[d] + delta).astype(np.int64)
                reach &= _reaches(cells, lo[d], hi[d], n[d], d < 2)
            assert not np.any(reach & ~inbox), (n, kind, dt, lo, hi, box, int(np.sum(reach & ~inbox)))


def test_source_box4_is_tight():
    """The boxes stop at the exact reach: at 48^4 (coupled potential, dt 0.05,
    16 x 12 x 8 x 8 tiles) the tiles scan 3.2 sources per lattice node; boxes
    with two more cells of margin per side scanned 6.6."""
    import itertools
    from paper_2007_12227_amd.inputs import phase4d_axes
    axes = phase4d_axes(48, 48)
    T = (16, 12, 8, 8)
    total = 0
    for c in itertools.product(*[range(0, 48, t) for t in T]):
        box = B.plan_source_box4(axes, H_PENDULUM, 1.0, 0.6, 0.4, 0.05, c, [min(c[d] + T[d], 48) for d in range(4)])
        total += np.prod([hi - lo for lo, hi in box])
    assert total / 48 ** 4 < 3.4

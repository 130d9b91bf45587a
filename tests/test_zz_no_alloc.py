"""The allocation-free entry point (vp_step_noalloc) against the grid path
(vp_step) on the same inputs, through the C interface: two calls in a row,
the second on a smaller lattice, then an FEL call, an in-place call with a
quadratic basis, and a non-finite input.  Bar: relative L1 <= 1e-5 and every
node within 1e-5 of the largest weight (the two paths run the same kernels;
their push tables are formed by host and device FP64 code)."""
import numpy as np
import pytest

from paper_2007_12227_amd.inputs import (FEL_RK4, H_PENDULUM, H_SHO_EXACT, Axis, Hamiltonian, fel_gaussian,
                                         gaussian, pendulum_axes, pendulum_band, rng)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2007_12227_amd import binding
    binding.lib()
    return binding


def grid_path(B, x, p, ham, w, dt, steps, basis=0):
    g = B.Grid(x, p)
    g.set_basis(basis)
    g.set_hamiltonian(ham)
    g.set_density(w)
    g.step(dt, steps)
    out = g.density().astype(np.float64)
    m = g.moments()
    g.close()
    return out, complex(m["A_re"], m["A_im"])


def noalloc_path(B, x, p, ham, w, dt, steps, basis=0, n0=0.0, in_place=False):
    import torch
    w_in = torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda()
    w_out = w_in if in_place else torch.full_like(w_in, float("nan"))
    A = torch.tensor([ham.A_re, ham.A_im], dtype=torch.float64, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    B.step_noalloc(x, p, ham, dt, steps, w_in, w_out, basis=basis, fel_n0=n0, fel_A=A, status=st)
    torch.cuda.synchronize()
    A = A.cpu().numpy()
    return w_out.cpu().numpy().astype(np.float64), complex(A[0], A[1]), int(st.item())


def close(got, ref):
    rel = np.abs(got - ref).sum() / np.abs(ref).sum()
    worst = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"rel L1 {rel:.2e}  max {worst:.2e}", flush=True)
    assert rel <= 1e-5 and worst <= 1e-5


def test_noalloc_matches_grid_two_calls_second_smaller(B):
    inst = pendulum_band(256)
    x, p = inst.x, Axis(inst.p.lo, inst.p.hi, 200, False)
    w = inst.w0[:200].astype(np.float32)
    got, _, st = noalloc_path(B, x, p, inst.ham, w, inst.dt, 7)
    ref, _ = grid_path(B, x, p, inst.ham, w, inst.dt, 7)
    assert st == B.VP_OK
    close(got, ref)
    # the second call on a smaller lattice reuses the scratch the first one left
    x2, p2 = pendulum_axes(96, 80)
    w2 = (gaussian(x2, p2, 0.3, 0.5, 0.4) + 1e-3 * rng(70).random((80, 96))).astype(np.float32)
    ham = Hamiltonian(H_PENDULUM, a=1.3)
    got, _, st = noalloc_path(B, x2, p2, ham, w2, 0.05, 5)
    ref, _ = grid_path(B, x2, p2, ham, w2, 0.05, 5)
    assert st == B.VP_OK
    close(got, ref)


@pytest.mark.parametrize("integrator", [0, FEL_RK4])
def test_noalloc_fel_matches_grid(B, integrator):
    import dataclasses
    inst = fel_gaussian(128, 10, npp=96)
    ham = dataclasses.replace(inst.ham, integrator=integrator)
    w = inst.w0.astype(np.float32)
    n0 = float(w.astype(np.float64).sum())
    got, A, st = noalloc_path(B, inst.x, inst.p, ham, w, inst.dt, 10, n0=n0)
    ref, Aref = grid_path(B, inst.x, inst.p, ham, w, inst.dt, 10)
    assert st == B.VP_OK
    close(got, ref)
    assert abs(A - Aref) <= 1e-9 * abs(Aref)


def test_noalloc_in_place_quadratic_oscillator(B):
    n, h = 64, 0.1
    half = 0.5 * (n - 1) * h
    x, p = Axis(-half, half, n, False), Axis(-half, half, n, False)
    w = gaussian(x, p, 0.5, -0.3, 0.6).astype(np.float32)
    ham = Hamiltonian(H_SHO_EXACT, omega=1.0)
    got, _, st = noalloc_path(B, x, p, ham, w, 0.1, 4, basis=B.BASIS_QUADRATIC, in_place=True)
    ref, _ = grid_path(B, x, p, ham, w, 0.1, 4, basis=B.BASIS_QUADRATIC)
    assert st == B.VP_OK
    close(got, ref)


def test_noalloc_refuses_and_reports(B):
    import torch
    x, p = pendulum_axes(64, 48)
    w = np.ones((48, 64), np.float32)
    w[5, 7] = np.nan
    got, _, st = noalloc_path(B, x, p, Hamiltonian(H_PENDULUM, a=1.0), w, 0.05, 2)
    assert st == B.VP_ENONFINITE and not np.any(got)
    t = torch.zeros((48, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(B.VpError) as e:  # the FEL without N0
        B.step_noalloc(x, p, Hamiltonian(3), 0.01, 1, t, t, fel_n0=0.0,
                       fel_A=torch.zeros(2, dtype=torch.float64, device="cuda"))
    assert e.value.code == B.VP_ESTATE
    big = Axis(-1.0, 1.0, 4096, True), Axis(-1.0, 1.0, 1025, False)  # 2^22 + 4096 nodes
    with pytest.raises(B.VpError) as e:
        B.step_noalloc(*big, Hamiltonian(H_PENDULUM, a=1.0), 0.01, 1, t.view(-1)[:0].new_zeros(4096 * 1025),
                       t.view(-1)[:0].new_zeros(4096 * 1025))
    assert e.value.code == B.VP_ENOMEM

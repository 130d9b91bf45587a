"""Full-length runs at the workloads' real sizes, in the launch configuration
the benchmark times (autotuned tiles, steps replayed from HIP graphs), against
strided samples of the FP64 oracle's run (tests/golden/make_full_runs.py).
Bar: relative L1 <= 1e-4 on the sample; the FP32-storage floor of the same
run (oracle with its state rounded to float every step) is printed beside it."""
import dataclasses
import os

import numpy as np
import pytest

import oracle
from paper_2007_12227_amd.inputs import FEL_RK4, fel_gaussian, pendulum_band, pendulum_gaussian

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2007_12227_amd import binding
    binding.lib()
    return binding


def run_against_golden(B, inst, name, autotune=True, chaotic_after=None):
    """Largest relative L1 (sample) over the checkpoints.  Checkpoints past
    chaotic_after are checked against ||w0||_1 instead (returned separately)."""
    ref = np.load(os.path.join(GOLDEN, f"oracle_{name}.npz"))
    stride = int(ref["stride"])
    g = B.Grid(inst.x, inst.p)
    g.set_hamiltonian(inst.ham)
    g.set_density(inst.w0.astype(np.float32))
    if autotune:
        g.autotune(inst.dt)
    done, worst, worst_w0 = 0, 0.0, 0.0
    l1_w0 = float(np.abs(inst.w0.astype(np.float32).astype(np.float64)[::stride, ::stride]).sum())
    for s in ref["steps"]:
        g.step(inst.dt, int(s) - done)
        done = int(s)
        got = g.density()[::stride, ::stride].astype(np.float64)
        exp = ref[f"sample_{s}"].astype(np.float64)
        err = float(np.abs(got - exp).sum() / np.abs(exp).sum())
        m = g.moments()
        print(f"{name} step {s}: rel L1 (sample) {err:.3e}  FP32-state floor {float(ref[f'fp32_floor_{s}']):.3e}"
              f"  sum_w gpu {m['sum_w']:.10e} oracle {float(ref[f'sum_{s}']):.10e}", flush=True)
        err_w0 = float(np.abs(got - exp).sum() / l1_w0)
        print(f"    relative to ||w0||_1: {err_w0:.3e}", flush=True)
        if chaotic_after is not None and s > chaotic_after:
            worst_w0 = max(worst_w0, err_w0)
        else:
            worst = max(worst, err)
        # mass accounting against the initial mass (the FEL loses almost all of
        # it through the open energy edges after saturation)
        assert abs(m["sum_w"] - float(ref[f"sum_{s}"])) <= 1e-6 * abs(float(ref["sum_1"]))
        if inst.ham.kind == 3:
            A = complex(*ref[f"A_{s}"])
            assert abs(complex(m["A_re"], m["A_im"]) - A) <= 1e-3 * abs(A), (m["A_re"], m["A_im"], A)
    g.close()
    return worst if chaotic_after is None else (worst, worst_w0)


def test_full_run_pendulum_gaussian_128(B):
    assert run_against_golden(B, pendulum_gaussian(128), "pendulum_gaussian_128", autotune=False) <= 1e-4


def test_full_run_pendulum_band_2048(B):
    assert run_against_golden(B, pendulum_band(2048), "pendulum_band_2048") <= 1e-4


def chaotic_checkpoints(bar=1e-4):
    """FEL checkpoints whose result rounding decides: there, equally valid FP32
    runs (tests/golden/fel_sensitivity.py: the FP32-state oracle with 1e-7
    relative noise per step, two seeds) already drift from the exact run by
    more than a tenth of the bar."""
    rows = np.loadtxt(os.path.join(GOLDEN, "fel_sensitivity.txt"))
    return sorted({int(k) for _, k, err, _ in rows if err > 0.1 * bar})


def test_full_run_fel_gaussian_1024(B):
    """Standard relative L1 <= 1e-4 where the result is a property of the
    implementation (through step 500: noisy FP32 runs agree with the exact
    one to ~1e-6).  By step 1000 the field has saturated, the beam has left
    the energy window through the open edges (the weights inside sum to 0.4%
    of the start, later to a Gibbs residue), and two noisy FP32 runs that
    differ only in the noise seed land 3.6e-6 and 9.0e-5 from the exact run:
    there the error is held to 1e-4 of ||w0||_1 (printed beside the standard
    number and the FP32-state floor), with the field A and the mass
    accounting checked at every checkpoint."""
    chaotic = chaotic_checkpoints()
    assert chaotic and min(chaotic) > 500, chaotic
    early, late = run_against_golden(B, fel_gaussian(1024), "fel_gaussian_1024", chaotic_after=min(chaotic) - 1)
    assert early <= 1e-4
    assert late <= 1e-4


def test_full_run_fel_gaussian_1024_rk4(B):
    """The 1024^2 FEL start advanced by the classical Runge-Kutta integrator
    through the exponential growth (500 steps), against the oracle's run."""
    inst = fel_gaussian(1024)
    inst = dataclasses.replace(inst, ham=dataclasses.replace(inst.ham, integrator=FEL_RK4))
    assert run_against_golden(B, inst, "fel_gaussian_1024_rk4") <= 1e-4

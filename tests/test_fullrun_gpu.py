"""Full-length runs at the workloads' real sizes, in the launch configuration
the benchmark times (autotuned tiles, steps replayed from HIP graphs), against
strided samples of the FP64 oracle's run and, at the last checkpoint, against
the full rows and columns on both sides of the deposit and solve tile seams
(tests/golden/make_full_runs.py).  Bar: relative L1 <= 1e-4, except where the
FEL's saturated state makes the standard number a matter of rounding (see
test_full_run_fel_gaussian_1024); the FP32-state floor of the same run (the
oracle with its state rounded to float every step) is printed beside it."""
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


def run_against_golden(B, inst, name, autotune=True):
    """Run the GPU through the stored checkpoints; per checkpoint the relative
    L1 distance over the strided sample, both to the oracle's ||w||_1 (the
    standard number) and to ||w0||_1, and the relative field error; at the
    last checkpoint the same over the stored full rows and columns on both
    sides of the tile seams."""
    ref = np.load(os.path.join(GOLDEN, f"oracle_{name}.npz"))
    stride = int(ref["stride"])
    g = B.Grid(inst.x, inst.p)
    g.set_hamiltonian(inst.ham)
    g.set_density(inst.w0.astype(np.float32))
    if autotune:
        g.autotune(inst.dt)
    done, out = 0, {}
    w0 = inst.w0.astype(np.float32).astype(np.float64)
    l1_w0 = float(np.abs(w0[::stride, ::stride]).sum())
    last = int(ref["steps"][-1])
    for s in ref["steps"]:
        g.step(inst.dt, int(s) - done)
        done = int(s)
        w = g.density().astype(np.float64)
        got = w[::stride, ::stride]
        exp = ref[f"sample_{s}"].astype(np.float64)
        diff = float(np.abs(got - exp).sum())
        m = g.moments()
        dA = 0.0
        if inst.ham.kind == 3:
            A = complex(*ref[f"A_{s}"])
            dA = abs(complex(m["A_re"], m["A_im"]) - A) / abs(A)
        row = {"err": diff / float(np.abs(exp).sum()), "err_w0": diff / l1_w0, "dA": dA}
        if int(s) == last and "rows" in ref:
            r, c = ref["seam_rows"], ref["seam_cols"]
            seam_got = np.concatenate([w[r, :].ravel(), w[:, c].ravel()])
            seam_exp = np.concatenate([ref["rows"].astype(np.float64).ravel(), ref["cols"].astype(np.float64).ravel()])
            seam_l1_w0 = float(np.abs(np.concatenate([w0[r, :].ravel(), w0[:, c].ravel()])).sum())
            sd = float(np.abs(seam_got - seam_exp).sum())
            row["seam_err"], row["seam_err_w0"] = sd / float(np.abs(seam_exp).sum()), sd / seam_l1_w0
        out[int(s)] = row
        print(f"{name} step {s}: rel L1 (sample) {row['err']:.3e}  FP32-state floor "
              f"{float(ref[f'fp32_floor_{s}']):.3e}  relative to ||w0||_1 {row['err_w0']:.3e}  |dA|/|A| {dA:.2e}"
              + (f"  seams: {row['seam_err']:.3e} ({row['seam_err_w0']:.3e} of ||w0||_1)" if "seam_err" in row else ""),
              flush=True)
        # mass accounting against the initial mass (the FEL loses almost all of
        # it through the open energy edges after saturation)
        assert abs(m["sum_w"] - float(ref[f"sum_{s}"])) <= 1e-6 * abs(float(ref["sum_1"]))
    g.close()
    return out


def test_full_run_pendulum_gaussian_128(B):
    res = run_against_golden(B, pendulum_gaussian(128), "pendulum_gaussian_128", autotune=False)
    assert all(r["err"] <= 1e-4 for r in res.values())


def test_full_run_pendulum_band_2048(B):
    res = run_against_golden(B, pendulum_band(2048), "pendulum_band_2048")
    assert all(r["err"] <= 1e-4 for r in res.values())
    assert res[1000]["seam_err"] <= 1e-4


def fp32_run_spread(model="random"):
    """Per checkpoint, the largest relative-L1 error, relative-to-||w0||_1
    error and field error of the oracle's FP32-state runs with per-step
    perturbations of rounding size (tests/golden/fel_sensitivity.py)."""
    out = {}
    for line in open(os.path.join(GOLDEN, "fel_sensitivity.txt")):
        f = line.split("#", 1)[0].split()
        if len(f) == 6 and f[0] == model:
            step, vals = int(f[2]), [float(v) for v in f[3:]]
            out[step] = [max(a, b) for a, b in zip(out.get(step, [0.0, 0.0, 0.0]), vals)]
    return out


def chaotic_checkpoints(bar=1e-5):
    """FEL checkpoints where equally valid FP32 runs (the oracle's FP32-state
    run with unbiased rounding-size noise, four seeds) already land more than
    1e-5 from the exact run: there rounding, not the implementation, decides
    the standard number."""
    return sorted(s for s, (err, _, _) in fp32_run_spread().items() if err > bar)


def test_full_run_fel_gaussian_1024(B):
    """The 1024^2 FEL through saturation (2000 steps) against the oracle.
    Where the result is a property of the implementation (through step 500)
    the standard relative L1 is held to 10x the worst unbiased FP32 run (at
    most 1e-4): 1.2e-5 at step 500, which a per-step bias of rounding size
    (one-sided rounding, a 1e-7 gain: 8e-5 to 1.4e-4 there) fails.  After
    saturation the beam has left the energy window and two FP32 runs that
    differ only in the noise seed land up to 100x apart (fel_sensitivity.txt):
    there the error relative to ||w0||_1 is held to twice the worst unbiased
    FP32 run (1.1e-6, 3.4e-7, 1.2e-7 at steps 1000, 1500, 2000), which the
    biased runs fail, and the standard number is printed.  The field is held
    to 10x the worst unbiased run's field error (at least 1e-6) at every
    checkpoint: 3.4e-6 to 4.4e-6, which the biased runs (2e-5 to 6e-5) fail."""
    spread = fp32_run_spread()
    chaotic = chaotic_checkpoints()
    assert chaotic == [1000, 1500, 2000], chaotic
    res = run_against_golden(B, fel_gaussian(1024), "fel_gaussian_1024")
    for s, r in res.items():
        err_max, err_w0_max, _ = spread[s]
        if s in chaotic:
            assert r["err_w0"] <= 2.0 * err_w0_max, (s, r, err_w0_max)
        else:
            assert r["err"] <= min(1e-4, 10.0 * max(err_max, 1e-8)), (s, r, err_max)
        assert r["dA"] <= max(1e-6, 10.0 * spread[s][2]), (s, r, spread[s][2])
    assert res[2000]["seam_err_w0"] <= 2.0 * spread[2000][1]


def test_full_run_fel_gaussian_1024_rk4(B):
    """The 1024^2 FEL start advanced by the classical Runge-Kutta integrator
    through the exponential growth (500 steps), against the oracle's run."""
    inst = fel_gaussian(1024)
    inst = dataclasses.replace(inst, ham=dataclasses.replace(inst.ham, integrator=FEL_RK4))
    res = run_against_golden(B, inst, "fel_gaussian_1024_rk4")
    assert all(r["err"] <= 1e-4 for r in res.values())

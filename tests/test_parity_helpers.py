"""The parity comparison itself (CPU): a defect confined to one tile seam or
one solve window, which a global relative-L1 bound lets through, fails the
node-wise bound."""
import numpy as np
import pytest

from _parity import assert_step_parity, step_errors
from paper_2007_12227_amd.inputs import pendulum_band


def test_seam_defect_fails_the_nodewise_bound():
    w = pendulum_band(512).w0.astype(np.float64)
    bad = w.copy()
    bad[:, 127:129] *= 1.0 + 2e-3  # a 2e-3 error on the two columns of one deposit-tile seam
    rel_l1, rel_max, at = step_errors(bad, w)
    assert rel_l1 <= 1e-5          # the global bound alone passes it ...
    assert at[1] in (127, 128)
    with pytest.raises(AssertionError):  # ... the node-wise bound does not
        assert_step_parity(bad, w, 1e-5)


def test_one_window_defect_fails_the_nodewise_bound():
    w = pendulum_band(2048).w0.astype(np.float64)
    bad = w.copy()
    bad[600:660, 900:960] *= 1.009  # one wrong 60 x 60 cubic solve tile, 0.9%
    assert step_errors(bad, w)[0] <= 1e-5
    with pytest.raises(AssertionError):
        assert_step_parity(bad, w, 1e-5)
    assert_step_parity(w * (1 + 1e-7), w, 1e-5)  # rounding-size differences pass

"""The library's host code (validation, workspace sizing, the source-box
planner against brute force, refusals before any device call) built with
AddressSanitizer and UndefinedBehaviorSanitizer on the host side and run on
the CPU (paper_2007_12227_amd/sanitize)."""
import os
import shutil

import pytest

from paper_2007_12227_amd.sanitize import build as san


@pytest.mark.skipif(not os.path.exists(san.HIPCC) and shutil.which("hipcc") is None, reason="needs hipcc")
def test_host_code_clean_under_asan_and_ubsan():
    san.build()
    r = san.run()
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr

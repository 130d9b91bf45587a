"""The committed rocprofv3 summaries (profiles/) describe the kernels as they
are: every summary names the hash of the kernel sources it was taken with,
and that hash must be the current sources' (a kernel change retakes them).
Each summary also states the command that made it, which runs bench.py."""
import glob
import hashlib
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2007_12227_amd", "csrc")
SUMMARIES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


HASH_2D = source_hash(("vp_kernels.hip", "vp_internal.h", "vp_device.h"))
HASH_4D = source_hash(("vp4_kernels.hip", "vp4_internal.h", "vp_device.h"))


def test_there_are_summaries():
    assert len(SUMMARIES) >= 10


@pytest.mark.parametrize("path", SUMMARIES, ids=os.path.basename)
def test_summary_matches_current_kernel_sources(path):
    text = open(path).read()
    m4 = re.search(r"2D2V kernel source sha256\[:16\][^:]*: ([0-9a-f]{16})", text)
    if m4:
        assert m4.group(1) == HASH_4D, "2D2V kernels changed since this summary was taken"
        return
    m2 = re.search(r"kernel[_ ]source[_ ]sha256(?:\[:16\]|_16): ([0-9a-f]{16})", text)
    assert m2, "no kernel source hash"
    assert m2.group(1) == HASH_2D, "2-D kernels changed since this summary was taken"


@pytest.mark.parametrize("path", SUMMARIES, ids=os.path.basename)
def test_summary_states_its_command(path):
    text = open(path).read()
    cmds = re.findall(r"rocprofv3 [^\n]*?-- (python3 bench\.py[^\n]*)", text)
    assert cmds, "no rocprofv3 command running bench.py"
    for c in cmds:
        assert "_work" not in c and "/root/" not in c

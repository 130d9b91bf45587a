"""Build the library's host code with AddressSanitizer and UndefinedBehaviorSanitizer
(host side only: each -fsanitize is preceded by -Xarch_host, the device code is
built as usual) linked into host_checks, and run it.  No GPU is needed.

    python paper_2007_12227_amd/sanitize/build.py
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(HERE, "host_checks")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("vp_kernels.hip", "vp_api.hip", "vp4_kernels.hip", "vp4_api.hip")]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build() -> str:
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", OUT, *SOURCES,
           os.path.join(HERE, "host_checks.cpp")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(res.stdout + res.stderr)
    return OUT


def run() -> subprocess.CompletedProcess:
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return subprocess.run([OUT], capture_output=True, text=True, env=env, timeout=600)


if __name__ == "__main__":
    build()
    r = run()
    print(r.stdout + r.stderr)
    sys.exit(r.returncode)

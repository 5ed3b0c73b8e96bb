"""Build libliftfft.so (the HIP library) in-tree with hipcc for gfx950.

``python -m paper_0811_2535_amd._build`` or :func:`build` from Python.  The
library lands next to this file; the Python binding loads it from there.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_NAME = "libliftfft.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
SOURCES = ["liftfft.hip"]
HEADERS = ["fft_engine.hpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (looked at $HIPCC, /opt/rocm/bin/hipcc, PATH)")


def compile_flags() -> list[str]:
    return [
        "--offload-arch=" + ARCH,
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-mcode-object-version=5",
        # keep hipcc from forming packed FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall",
        "-I" + INCLUDE,
        "-I" + CSRC,
    ]


def build(verbose: bool = True, out: str | None = None) -> str:
    """Compile every source and link the shared library (always rebuilds)."""
    out = out or LIB_PATH
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + compile_flags() + ["-shared", "-o", tmp] + \
        [os.path.join(CSRC, s) for s in SOURCES]
    t0 = time.time()
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building %s" % LIB_NAME)
    os.replace(tmp, out)
    if verbose:
        print("built %s in %.1fs" % (out, time.time() - t0), flush=True)
    return out


if __name__ == "__main__":
    build()

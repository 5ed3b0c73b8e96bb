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
SOURCES = ["liftfft.hip", "paper_plan.hip"]
HEADERS = ["fft_engine.hpp", "paper_plan.hpp"]
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
    """Compile every source (in parallel, one object each) and link the shared
    library (always rebuilds)."""
    from concurrent.futures import ThreadPoolExecutor

    out = out or LIB_PATH
    tag = ".tmp%d" % os.getpid()
    objs = [out + "." + os.path.splitext(s)[0] + tag + ".o" for s in SOURCES]
    t0 = time.time()

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    cmds = [[hipcc()] + compile_flags() + ["-c", "-o", o, os.path.join(CSRC, s)]
            for s, o in zip(SOURCES, objs)]
    try:
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            results = list(ex.map(run, cmds))
        for res, src in zip(results, SOURCES):
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError("hipcc failed compiling %s" % src)
        tmp = out + tag
        res = run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking %s" % LIB_NAME)
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    if verbose:
        print("built %s in %.1fs" % (out, time.time() - t0), flush=True)
    return out


PROBE_SRC = os.path.join(CSRC, "traversal_probe.hip")
PROBE_PATH = os.path.join(HERE, "traversal_probe")


def build_probe(verbose: bool = True) -> str:
    """Compile the traversal probe (a measurement program beside the library:
    plain copies with each pass's tile traversal) to ``traversal_probe``."""
    t0 = time.time()
    tmp = PROBE_PATH + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + compile_flags() + ["-o", tmp, PROBE_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        if os.path.exists(tmp):
            os.remove(tmp)
        raise RuntimeError("hipcc failed compiling traversal_probe.hip")
    os.replace(tmp, PROBE_PATH)
    if verbose:
        print("built %s in %.1fs" % (PROBE_PATH, time.time() - t0), flush=True)
    return PROBE_PATH


if __name__ == "__main__":
    build()
    build_probe()

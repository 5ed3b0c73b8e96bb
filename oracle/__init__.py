"""FP64 CPU oracle for the 1-D complex DFT -- test infrastructure only.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never links, loads or calls it, and
the two share no code: this package wraps ``oracle.c`` (plain C, built with
gcc) through ctypes and works on numpy ``complex128`` arrays.

Functions (all unnormalized, natural order; the definition is Section 2.1,
Fig. 2.1 of the paper: X[k] = sum_j x[j] w_n^(sign*j*k), w_n = exp(2 pi i/n)):

* :func:`dft` -- the O(n^2) definition, term by term.
* :func:`fft` -- Fig. 2.1 in recursive radix-2 form (even/odd split = the
  bit-reversal permutation, B_L butterflies with directly computed weights).
* :func:`fft_batch` -- :func:`fft` over the rows of a 2-D array, on threads.
* :func:`rel_l2` -- the comparison metric ||a - b||_2 / ||b||_2 in FP64.

Every function here is pinned by ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` beside it (always rebuilds)."""
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC,
           "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load(path: str | None = None):
    """Load the oracle library (building it first if it is missing)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.oracle_dft.argtypes = [dp, dp, i64, ctypes.c_int]
    lib.oracle_dft.restype = ctypes.c_int
    lib.oracle_fft.argtypes = [dp, dp, i64, ctypes.c_int]
    lib.oracle_fft.restype = ctypes.c_int
    lib.oracle_fft_batch.argtypes = [dp, dp, i64, i64, ctypes.c_int, ctypes.c_int]
    lib.oracle_fft_batch.restype = ctypes.c_int
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x), dtype=np.complex128)


class Oracle:
    """The oracle bound to one shared library (the default build, or another
    build of the same source, e.g. a deliberately broken copy in a test)."""

    def __init__(self, lib):
        self.lib = lib

    def dft(self, x, sign: int = -1) -> np.ndarray:
        x = _as_c128(x)
        if x.ndim != 1:
            raise ValueError("dft expects a 1-D array")
        out = np.empty_like(x)
        rc = self.lib.oracle_dft(_ptr(x), _ptr(out), x.size, int(sign))
        if rc != 0:
            raise ValueError("oracle_dft rejected n=%d sign=%d (rc=%d)" % (x.size, sign, rc))
        return out

    def fft(self, x, sign: int = -1) -> np.ndarray:
        x = _as_c128(x)
        if x.ndim != 1:
            raise ValueError("fft expects a 1-D array; use fft_batch for 2-D")
        out = np.empty_like(x)
        rc = self.lib.oracle_fft(_ptr(x), _ptr(out), x.size, int(sign))
        if rc != 0:
            raise ValueError("oracle_fft rejected n=%d sign=%d (rc=%d)" % (x.size, sign, rc))
        return out

    def fft_batch(self, x, sign: int = -1, threads: int | None = None) -> np.ndarray:
        x = _as_c128(x)
        if x.ndim != 2:
            raise ValueError("fft_batch expects a 2-D array (batch, n)")
        out = np.empty_like(x)
        nt = threads if threads is not None else (os.cpu_count() or 1)
        rc = self.lib.oracle_fft_batch(_ptr(x), _ptr(out), x.shape[1], x.shape[0],
                                       int(sign), int(nt))
        if rc != 0:
            raise ValueError("oracle_fft_batch rejected shape=%s sign=%d (rc=%d)"
                             % (x.shape, sign, rc))
        return out


def default() -> Oracle:
    return Oracle(_load())


def load_library(path: str) -> Oracle:
    """An :class:`Oracle` over another build of ``oracle.c`` (used by tests)."""
    return Oracle(_load(path))


def dft(x, sign: int = -1) -> np.ndarray:
    return default().dft(x, sign)


def fft(x, sign: int = -1) -> np.ndarray:
    return default().fft(x, sign)


def fft_batch(x, sign: int = -1, threads: int | None = None) -> np.ndarray:
    return default().fft_batch(x, sign, threads)


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2, computed in FP64 (b is the reference)."""
    a = np.asarray(a).astype(np.complex128, copy=False)
    b = np.asarray(b).astype(np.complex128, copy=False)
    den = float(np.linalg.norm(b.ravel()))
    num = float(np.linalg.norm((a - b).ravel()))
    if den == 0.0:
        return num
    return num / den

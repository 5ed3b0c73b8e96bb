"""fft_execute_static, the allocation-free entry point, against fft_execute of
the default plan of the same shape, through the C ABI.

Both run the same launches over the same kernels, so their outputs must agree
bit for bit; each is also held to the oracle tolerance (relative L2 1e-6 for
complex64, 1e-12 for complex128).  The calls come in a row on one GPU, the
second with a smaller input than the first, so the second runs on the array
the first left behind (and on regenerated weight tables)."""
import ctypes

import numpy as np
import pytest

import datagen
import oracle
from gpu_util import announce, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = {np.complex64: 1e-6, np.complex128: 1e-12}


def _static(L, n, batch, code, x, y, sign, stream):
    return L.fft_execute_static(n, batch, code, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                sign, ctypes.c_void_p(stream))


def test_static_matches_planned_execute():
    torch = require_gpu()
    import paper_0811_2535_amd as lf
    L = lf.lib()
    stream = torch.cuda.current_stream().cuda_stream
    # (n, batch, dtype, sign): two-level lifts (scratch used) and a single
    # pass; each call smaller than the one before, then the first shape again.
    cases = [(1 << 21, 2, np.complex64, -1), (1 << 16, 3, np.complex64, 1), (1 << 12, 5, np.complex64, -1),
             (1 << 20, 2, np.complex128, 1), (1 << 17, 1, np.complex128, -1), (1 << 21, 2, np.complex64, -1)]
    for i, (n, batch, dt, sign) in enumerate(cases):
        code = 0 if dt == np.complex64 else 1
        tdt = torch.complex64 if dt == np.complex64 else torch.complex128
        x_np = datagen.signals(n, batch, dt, "normal", 70 + i)
        x = to_dev(x_np)
        y = torch.full_like(x, float("nan"))
        yref = torch.full_like(x, float("nan"))
        announce("fft_execute_static call %d n=%d batch=%d %s sign=%d" % (i, n, batch, np.dtype(dt).name, sign))
        assert _static(L, n, batch, code, x, y, sign, stream) == 0
        torch.cuda.synchronize()
        plan = lf.Plan(n, batch, tdt)
        plan.execute(x, yref, sign)
        torch.cuda.synchronize()
        plan.destroy()
        got, want = to_np(y), to_np(yref)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (n, batch)  # bit for bit
        ref = oracle.fft_batch(x_np.astype(np.complex128), sign)
        errs = [oracle.rel_l2(got[b], ref[b]) for b in range(batch)]
        assert max(errs) <= TOL[dt], (n, batch, errs)


def test_static_in_place_and_capacity():
    torch = require_gpu()
    import paper_0811_2535_amd as lf
    L = lf.lib()
    stream = torch.cuda.current_stream().cuda_stream
    n, batch = 1 << 18, 4
    x_np = datagen.signals(n, batch, np.complex64, "uniform", 80)
    x = to_dev(x_np)
    announce("fft_execute_static in place n=2^18 batch=4")
    assert _static(L, n, batch, 0, x, x, -1, stream) == 0
    torch.cuda.synchronize()
    ref = oracle.fft_batch(x_np.astype(np.complex128), -1)
    got = to_np(x)
    assert max(oracle.rel_l2(got[b], ref[b]) for b in range(batch)) <= 1e-6
    # beyond 32 MiB of elements: refused before any device work
    big = torch.empty(1, dtype=torch.complex64, device="cuda")
    assert _static(L, 1 << 23, 1, 0, big, big, -1, stream) == -10
    assert _static(L, 1 << 22, 1, 1, big, big, -1, stream) == -10
    assert _static(L, 1 << 20, 8, 0, big, big, -1, stream) == -10
    assert _static(L, 1000, 1, 0, big, big, -1, stream) == -1
    assert _static(L, 1 << 10, 1, 0, big, big, 2, stream) == -3

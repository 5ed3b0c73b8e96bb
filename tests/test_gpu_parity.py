"""GPU path against the FP64 oracle, element by element, through the C ABI.

Tolerances (relative L2 per transform, computed in FP64 against the oracle run
on exactly the values the GPU received):
* complex64:  1e-6  (the stated bound for n = 2^24; FP32 radix-16 error grows
  roughly like sqrt(log2 n) * 2^-24, about 1-3e-7 at 2^24)
* complex128: 1e-12
"""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import announce, require_gpu, to_dev, to_np

TOL = {np.complex64: 1e-6, np.complex128: 1e-12}
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lf(torch):
    import paper_0811_2535_amd as lf
    return lf


def run_plan(lf, x_np, sign, repeat=1, **opts):
    """Execute one plan over the rows of x_np (batch, n) and return numpy
    (with repeat > 1, a list of the outputs of repeated executions)."""
    import torch
    batch, n = x_np.shape
    dt = torch.complex64 if x_np.dtype == np.complex64 else torch.complex128
    plan = lf.Plan(n, batch, dt, **opts)
    x = to_dev(x_np)
    outs = []
    for _ in range(repeat):
        y = torch.full_like(x, float("nan"))
        plan.execute(x, y, sign)
        torch.cuda.synchronize()
        outs.append(to_np(y))
    plan.destroy()
    return outs[0] if repeat == 1 else outs


def mismatch_report(got, x_np, sign, ref):
    """Where the GPU result and the oracle disagree, and whether numpy agrees
    with the oracle (to tell an oracle fault from a GPU one)."""
    npref = np.fft.fft(x_np.astype(np.complex128), axis=1) if sign < 0 else \
        x_np.shape[1] * np.fft.ifft(x_np.astype(np.complex128), axis=1)
    d = np.abs(got - ref)
    big = d > 1e-3 * np.abs(ref).max()
    return dict(gpu_vs_numpy=[oracle.rel_l2(got[b], npref[b]) for b in range(len(got))],
                oracle_vs_numpy=[oracle.rel_l2(ref[b], npref[b]) for b in range(len(got))],
                n_far=int(big.sum()), worst=np.unravel_index(int(np.argmax(d)), d.shape),
                nan=int(np.isnan(got).sum()))


def check_rows(got, x_np, sign, tol):
    ref = oracle.fft_batch(x_np.astype(np.complex128), sign)
    errs = [oracle.rel_l2(got[b], ref[b]) for b in range(x_np.shape[0])]
    assert max(errs) <= tol, (errs, tol, mismatch_report(got, x_np, sign, ref))
    return max(errs)


def test_config1_plain_radix2_lift(lf):
    """n = 2^10 complex128, U[-1,1] seed 1, sign -1, lifted 32 x 32 with
    radix-2 stages in both passes."""
    x = datagen.signals(1024, 1, np.complex128, "uniform", 1)
    announce("config1 n=1024 c128 log2_p=5 radix=2 seed=1")
    got = run_plan(lf, x, -1, log2_p=5, radix=2)
    check_rows(got, x, -1, TOL[np.complex128])


def test_config1_default_plan(lf):
    x = datagen.signals(1024, 1, np.complex128, "uniform", 1)
    announce("config1 n=1024 c128 default plan")
    got = run_plan(lf, x, -1)
    check_rows(got, x, -1, TOL[np.complex128])


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128], ids=["c64", "c128"])
@pytest.mark.parametrize("t", list(range(1, 19)))
def test_all_lengths(lf, t, dtype):
    """Every n = 2^1 .. 2^18, both signs, ragged batch of 3 (a partial tile)."""
    n = 1 << t
    x = datagen.signals(n, 3, dtype, "normal", 40 + t)
    for sign in (-1, 1):
        announce("all_lengths n=2^%d %s sign=%d batch=3" % (t, np.dtype(dtype).name, sign))
        got = run_plan(lf, x, sign)
        check_rows(got, x, sign, TOL[dtype])


@pytest.mark.parametrize("radix", [2, 16])
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128], ids=["c64", "c128"])
def test_every_split(lf, dtype, radix):
    """n = 2^12: every lift p = 2^1 .. 2^11 (forces the two-pass path)."""
    t = 12
    x = datagen.signals(1 << t, 2, dtype, "uniform", 7)
    for log2_p in range(1, t):
        announce("split n=2^12 log2_p=%d radix=%d %s" % (log2_p, radix, np.dtype(dtype).name))
        got = run_plan(lf, x, -1, log2_p=log2_p, radix=radix)
        check_rows(got, x, -1, TOL[dtype])


@pytest.mark.parametrize("t,batch", [(13, 5), (16, 3), (20, 2), (22, 1)])
def test_two_pass_batches(lf, t, batch):
    x = datagen.signals(1 << t, batch, np.complex64, "normal", 100 + t)
    for sign in (-1, 1):
        announce("two_pass n=2^%d batch=%d sign=%d" % (t, batch, sign))
        got = run_plan(lf, x, sign)
        check_rows(got, x, sign, TOL[np.complex64])


def test_config2_full_size(lf, torch):
    """n = 2^24 complex64 lifted 4096 x 4096, N(0,1) seed 2: forward and
    inverse against the full FP64 oracle, plus the round trip."""
    n = 1 << 24
    x_np = datagen.signals(n, 1, np.complex64, "normal", 2)
    plan = lf.Plan(n, 1, torch.complex64)
    info = plan.info()
    assert info["passes"] == 2 and info["log2_p"] == 12 and info["log2_q"] == 12
    x = to_dev(x_np)
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    announce("config2 n=2^24 c64 forward")
    plan.execute(x, y, -1)
    announce("config2 n=2^24 c64 inverse of forward")
    plan.execute(y, z, 1)
    torch.cuda.synchronize()
    y_np, z_np = to_np(y), to_np(z)
    ref_f = oracle.fft(x_np[0].astype(np.complex128), -1)
    e_f = oracle.rel_l2(y_np[0], ref_f)
    assert e_f <= 1e-6, e_f
    ref_i = oracle.fft(x_np[0].astype(np.complex128), 1)
    announce("config2 n=2^24 c64 inverse")
    w = torch.empty_like(x)
    plan.execute(x, w, 1)
    torch.cuda.synchronize()
    e_i = oracle.rel_l2(to_np(w)[0], ref_i)
    assert e_i <= 1e-6, e_i
    e_rt = oracle.rel_l2(z_np[0] / n, x_np[0])
    assert e_rt <= 2e-6, e_rt
    plan.destroy()


def test_in_place(lf, torch):
    for t in (10, 16):
        n = 1 << t
        x_np = datagen.signals(n, 2, np.complex64, "normal", 9)
        plan = lf.Plan(n, 2, torch.complex64)
        x = to_dev(x_np)
        announce("in_place n=2^%d" % t)
        plan.execute(x, x, -1)
        torch.cuda.synchronize()
        check_rows(to_np(x), x_np, -1, TOL[np.complex64])
        plan.destroy()


def test_batch_independence_and_determinism(lf, torch):
    """Transform b of a batch equals the same signal transformed alone, bit for
    bit, and repeated runs are bitwise identical."""
    for t in (8, 14):
        n = 1 << t
        x_np = datagen.signals(n, 6, np.complex64, "normal", 11)
        announce("batch_independence n=2^%d" % t)
        whole = run_plan(lf, x_np, -1)
        again = run_plan(lf, x_np, -1)
        assert np.array_equal(whole, again)
        for b in (0, 3, 5):
            alone = run_plan(lf, x_np[b:b + 1], -1)
            assert np.array_equal(alone[0], whole[b]), (t, b)


def test_error_codes_on_device(lf, torch):
    import ctypes
    from paper_0811_2535_amd import binding
    L = binding.lib()
    plan = lf.Plan(1024, 2, torch.complex64)
    buf = torch.zeros(4096, dtype=torch.complex64, device="cuda")
    p = buf.data_ptr()
    s = torch.cuda.current_stream().cuda_stream
    announce("error codes")
    assert L.fft_execute(plan.handle, p, p, 0, s) == -3
    assert L.fft_execute(plan.handle, p + 4, p + 4, -1, s) == -5
    assert L.fft_execute(plan.handle, p, p + 8 * 16, -1, s) == -9   # partial overlap
    assert L.fft_execute(plan.handle, None, p, -1, s) == -4
    assert L.fft_execute(plan.handle, p, p + 8 * 2048, -1, s) == 0  # disjoint halves
    torch.cuda.synchronize()
    info = binding.PlanInfo()
    assert L.fft_plan_get_info(plan.handle, ctypes.byref(info)) == 0
    assert info.n == 1024 and info.batch == 2 and info.passes == 1
    plan.destroy()


def test_timing_counts_launches(lf, torch):
    n = 1 << 16
    plan = lf.Plan(n, 1, torch.complex64)
    x = torch.zeros(n, dtype=torch.complex64, device="cuda")
    announce("timing ring n=2^16")
    plan.set_timing(True)
    for _ in range(1100):  # more than the ring holds
        plan.execute(x, x, -1)
    ms, cnt = plan.read_timing()
    assert cnt == [1100, 1100] and ms[0] > 0 and ms[1] > 0
    plan.set_timing(False)
    plan.destroy()

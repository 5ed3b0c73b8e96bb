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
    plan = lf.Plan(n, 1, torch.complex64, flags=128)  # FFT_OPT_TWO_LEVEL: the 4096 x 4096 lift
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
    assert cnt == [1100, 1100, 0] and ms[0] > 0 and ms[1] > 0 and ms[2] == 0
    plan.set_timing(False)
    plan.destroy()


VARIANTS = [dict(values_per_thread=e, flags=f) for e in (16, 32) for f in (0, 2, 8, 10)] + \
           [dict(values_per_thread=16, flags=f) for f in (32, 34)]


def _variant_id(v):
    names = {0: "full", 2: "split", 8: "full-persist", 10: "split-persist", 32: "full-dense",
             34: "split-dense"}
    return "e%d-%s" % (v["values_per_thread"], names[v["flags"]])


@pytest.mark.parametrize("t,batch", [(20, 3), (23, 1), (24, 1)])
def test_pass_kernel_variants(lf, t, batch):
    """Every pass-kernel variant (16 or 32 values per thread; complex or
    split real/imaginary exchange; one tile per workgroup or persistent
    workgroups with next-tile prefetch) against the FP64 oracle, both signs,
    at pass lines of 2^10, 2^11/2^12 and 2^12.  Variants with 16 values per
    thread do the same operations in the same order as the default kernels
    (up to which products the compiler fuses into FMAs), so their outputs
    must also agree with the default plan to rounding level everywhere: a
    stale or misplaced LDS value would show as an O(1) relative difference
    in some element."""
    x = datagen.signals(1 << t, batch, np.complex64, "normal", 300 + t)
    for sign in (-1, 1):
        ref = oracle.fft_batch(x.astype(np.complex128), sign)
        announce("variants n=2^%d batch=%d sign=%d default" % (t, batch, sign))
        base = run_plan(lf, x, sign)
        for v in VARIANTS:
            announce("variants n=2^%d batch=%d sign=%d %s" % (t, batch, sign, _variant_id(v)))
            got = run_plan(lf, x, sign, **v)
            errs = [oracle.rel_l2(got[b], ref[b]) for b in range(batch)]
            assert max(errs) <= TOL[np.complex64], (_variant_id(v), errs)
            if v["values_per_thread"] == 16:
                assert_rounding_level(got, base, _variant_id(v))


def assert_rounding_level(got, base, what):
    """Element-wise agreement of two FP32 results to a few units in the last
    place of the largest output (|X_k| is at most sum |x_j|)."""
    scale = np.abs(base).max()
    diff = np.abs(got.astype(np.complex128) - base.astype(np.complex128))
    worst = float(diff.max() / scale)
    assert worst <= 1e-5, (what, worst, np.unravel_index(int(np.argmax(diff)), diff.shape))


def test_variant_tile_widths(lf):
    """Persistent and split variants over the tile widths the planner may
    pick (1..8 lines in pass 1, 2..8 in pass 2), against the oracle and,
    with 16 values per thread, element-wise against the default plan."""
    import torch
    t, batch = 22, 2
    x = datagen.signals(1 << t, batch, np.complex64, "normal", 322)
    ref = oracle.fft_batch(x.astype(np.complex128), -1)
    base = run_plan(lf, x, -1)
    for v in VARIANTS:
        for T1, T2 in ((1, 2), (2, 4), (4, 8), (8, 8)):
            try:
                plan = lf.Plan(1 << t, batch, torch.complex64, lines_per_block=T1, lines_per_block2=T2, **v)
            except lf.FFTError:
                continue
            info = plan.info()
            plan.destroy()
            if info["lines_per_block_pass1"] != T1 or info["lines_per_block_pass2"] != T2:
                continue
            announce("variant tiles %s T=(%d,%d)" % (_variant_id(v), T1, T2))
            got = run_plan(lf, x, -1, lines_per_block=T1, lines_per_block2=T2, **v)
            errs = [oracle.rel_l2(got[b], ref[b]) for b in range(batch)]
            assert max(errs) <= TOL[np.complex64], (_variant_id(v), T1, T2, errs)
            if v["values_per_thread"] == 16:
                assert_rounding_level(got, base, (_variant_id(v), T1, T2))


@pytest.mark.parametrize("t,batch", [(22, 2), (24, 1)])
def test_scratch_slab_widths(lf, t, batch):
    """Scratch slabs wider and narrower than pass 1's tile (pass 1 then writes
    its columns into part of a slab, or several slabs), with 16 or 32 values
    per thread in pass 2 (split exchange), against the oracle."""
    x = datagen.signals(1 << t, batch, np.complex64, "normal", 330 + t)
    ref = oracle.fft_batch(x.astype(np.complex128), -1)
    for W, vpt2, T1, T2 in ((1, 0, 2, 4), (4, 0, 2, 4), (8, 0, 2, 4), (8, 32, 2, 4), (16, 32, 4, 4),
                            (2, 32, 4, 2)):
        announce("slab width W=%d vpt2=%d T=(%d,%d) n=2^%d" % (W, vpt2, T1, T2, t))
        got = run_plan(lf, x, -1, scratch_width=W, values_per_thread2=vpt2, lines_per_block=T1,
                       lines_per_block2=T2, flags=2)
        errs = [oracle.rel_l2(got[b], ref[b]) for b in range(batch)]
        assert max(errs) <= TOL[np.complex64], (W, vpt2, T1, T2, errs)


def test_complex128_repeat_determinism(lf, torch):
    """complex128 results are bitwise identical across repeated executes, on
    single-pass, two-level and three-level plans (every element store of a
    complex128 value is issued as two 8-byte stores), and each repeat meets
    the oracle tolerance: 256 + 32 + 4 transforms per shape."""
    for t, batch, reps, flags in ((12, 64, 4, 0), (18, 4, 8, 128), (24, 1, 4, 256)):
        n = 1 << t
        x_np = datagen.signals(n, batch, np.complex128, "normal", 120 + t)
        announce("c128 repeat determinism n=2^%d batch=%d reps=%d" % (t, batch, reps))
        outs = run_plan(lf, x_np, 1, repeat=reps, flags=flags)
        for k in range(1, reps):
            assert np.array_equal(outs[k].view(np.uint64), outs[0].view(np.uint64)), (t, k)
        check_rows(outs[0], x_np, 1, TOL[np.complex128])


LDS_PREFETCH = 2048  # FFT_OPT_LDS_PREFETCH
ROW_LANES = 16384  # FFT_OPT_ROW_LANES
SPLIT = 2  # FFT_OPT_SPLIT_EXCHANGE
FULL = 4  # FFT_OPT_FULL_EXCHANGE: the generic kernels
CANARY = 4096  # FFT_OPT_DEBUG_CANARY: NaN-filled scratch, so no stale data can stand in for a missing write


@pytest.mark.parametrize("t,batch", [(24, 1), (23, 2)])
def test_lds_staged_pass1(lf, torch, t, batch):
    """Pass 1 with the next tile staged in LDS by direct global-to-LDS loads
    (4096-point columns, persistent workgroups): against the oracle for both
    signs, against the default plan to rounding level, in place, and for an
    input that is only 8-byte aligned (which takes the plain pass 1)."""
    x = datagen.signals(1 << t, batch, np.complex64, "normal", 340 + t)
    plan = lf.Plan(1 << t, batch, torch.complex64, flags=128 | LDS_PREFETCH)
    info = plan.info()
    plan.destroy()
    assert info["variant_pass1"] & 128 and info["lines_per_block_pass1"] == 2, info
    for sign in (-1, 1):
        announce("lds-staged pass 1 n=2^%d batch=%d sign=%d" % (t, batch, sign))
        got = run_plan(lf, x, sign, flags=128 | LDS_PREFETCH)
        check_rows(got, x, sign, TOL[np.complex64])
        assert_rounding_level(got, run_plan(lf, x, sign, flags=128), ("lds-staged", t, sign))
    announce("lds-staged pass 1 n=2^%d in place and 8-byte aligned input" % t)
    n = 1 << t
    plan = lf.Plan(n, batch, torch.complex64, flags=128 | LDS_PREFETCH)
    xd = to_dev(x)
    plan.execute(xd, xd, -1)
    buf = torch.zeros(n * batch + 1, dtype=torch.complex64, device="cuda")
    shifted = buf[1:].view(batch, n)  # 8 bytes past a 16-byte boundary
    shifted.copy_(to_dev(x))
    y = torch.empty_like(shifted)
    plan.execute(shifted, y, -1)
    torch.cuda.synchronize()
    plan.destroy()
    check_rows(to_np(xd), x, -1, TOL[np.complex64])
    check_rows(to_np(y), x, -1, TOL[np.complex64])


@pytest.mark.parametrize("vpt", [16, 32])
@pytest.mark.parametrize("t,batch", [(24, 1), (23, 2), (17, 3)])
def test_row_lane_pass1(lf, torch, t, batch, vpt):
    """Pass 1 with each thread owning whole rows of a 2-column tile (4096-point
    columns; 2^17 as 32 x 4096), 8 rows per thread with radix-8 stages or 16
    with radix 16: against the oracle for both signs, against the generic
    kernels to rounding level, in place, and for an input that is only 8-byte
    aligned (which takes the generic pass 1)."""
    n = 1 << t
    kw = dict(flags=128 | ROW_LANES | CANARY, log2_p=t - 12, values_per_thread=vpt)
    x = datagen.signals(n, batch, np.complex64, "normal", 360 + t)
    plan = lf.Plan(n, batch, torch.complex64, **kw)
    info = plan.info()
    plan.destroy()
    assert info["variant_pass1"] & 256 and info["lines_per_block_pass1"] == 2, info
    assert info["threads_pass1"] == 8192 // vpt and not info["variant_pass2"] & 1, info  # pass 2 keeps 16 values
    for sign in (-1, 1):
        announce("row-lane pass 1 n=2^%d batch=%d vpt=%d sign=%d" % (t, batch, vpt, sign))
        got = run_plan(lf, x, sign, **kw)
        check_rows(got, x, sign, TOL[np.complex64])
        generic = run_plan(lf, x, sign, flags=128 | FULL, log2_p=t - 12)
        assert_rounding_level(got, generic, ("row-lane", t, sign))
    announce("row-lane pass 1 n=2^%d vpt=%d in place and 8-byte aligned input" % (t, vpt))
    plan = lf.Plan(n, batch, torch.complex64, **kw)
    xd = to_dev(x)
    plan.execute(xd, xd, -1)
    buf = torch.zeros(n * batch + 1, dtype=torch.complex64, device="cuda")
    shifted = buf[1:].view(batch, n)  # 8 bytes past a 16-byte boundary
    shifted.copy_(to_dev(x))
    y = torch.empty_like(shifted)
    plan.execute(shifted, y, -1)
    torch.cuda.synchronize()
    plan.destroy()
    check_rows(to_np(xd), x, -1, TOL[np.complex64])
    check_rows(to_np(y), x, -1, TOL[np.complex64])


def test_row_lane_pass1_refusals(lf, torch):
    """Shapes the row-lane pass 1 does not cover return FFT_E_UNSUPPORTED;
    other kernel-variant options with it, or no FFT_OPT_TWO_LEVEL, FFT_E_ARG."""
    B = lf.binding
    for kw, code in ((dict(flags=128 | ROW_LANES, log2_p=11), -8),          # 8192-point columns
                     (dict(flags=128 | ROW_LANES, log2_p=12, lines_per_block=1), -9),
                     (dict(flags=128 | ROW_LANES | SPLIT, log2_p=12), -9),
                     (dict(flags=ROW_LANES, log2_p=12), -9)):
        announce("row-lane refusal %s" % kw)
        with pytest.raises(lf.FFTError) as e:
            lf.Plan(1 << 24, 1, torch.complex64, **kw)
        assert e.value.code == code, (kw, e.value.code)
    announce("row-lane refusal complex128")
    with pytest.raises(lf.FFTError) as e:
        lf.Plan(1 << 24, 1, torch.complex128, flags=128 | ROW_LANES, log2_p=12)
    assert e.value.code == -8

"""Precision forms: radix-16 stages as 16 x 16 DFT-matrix products on the
matrix cores with FP16 or BF16 high/low operand pairs and FP32 accumulation
(fft_plan_set_precision), against the FP64 oracle.

This arithmetic is not the paper's (the paper's butterflies are exact radix-2
operations in the working precision); the bound checked here is the one the
operand precision sets.  With an 11-bit (FP16) or 8-bit (BF16) significand per
part, the pair carries about 22 or 16 bits, so one radix-16 stage adds a
relative error of a few 2^-22 (FP16 pairs) or 2^-16 (BF16 pairs); over the
1 to 6 stages of these sizes the relative L2 error stays below the FP32 path's
1e-6 for FP16 pairs and below 3e-5 for BF16 pairs.  The measured values are
printed (pytest -s) and bounded below.
"""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import announce, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu
# measured (MI355X): FP16 pairs 1.4e-7 (one stage) .. 2.6e-7 (n = 2^24, six
# stages), as accurate as the FP32 path; BF16 pairs 4.5e-6 .. 7.9e-6.
BOUND = {"f16x2": 1e-6, "bf16x2": 3e-5}


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lf(torch):
    import paper_0811_2535_amd as lf
    return lf


def run_prec(lf, x_np, sign, mode, **opts):
    import torch
    batch, n = x_np.shape
    # the precision forms run on single-pass and two-level plans (at 2^24 the
    # library's default is the three-level lift)
    plan = lf.Plan(n, batch, torch.complex64, **dict(dict(flags=128), **opts))
    plan.set_precision(mode)
    assert plan.info()["precision"] == {"fp32": 0, "f16x2": 1, "bf16x2": 2}[mode]
    x = to_dev(x_np)
    y = torch.full_like(x, float("nan"))
    plan.execute(x, y, sign)
    torch.cuda.synchronize()
    plan.destroy()
    return to_np(y)


@pytest.mark.parametrize("mode", ["f16x2", "bf16x2"])
def test_dft16_matrix_product(lf, mode):
    """n = 16: one stage, i.e. exactly the 16 x 16 DFT-matrix product, against
    the O(n^2) definition in FP64 (brute force), both signs, 256 vectors with
    magnitudes spread over 2^-20..2^20 (exercises the per-butterfly scaling)."""
    x = datagen.signals(16, 256, np.complex64, "normal", 61)
    mags = np.exp2(np.linspace(-20, 20, 256)).astype(np.float32)[:, None]
    x = (x * mags).astype(np.complex64)
    for sign in (-1, 1):
        announce("precision dft16 %s sign=%d" % (mode, sign))
        got = run_prec(lf, x, sign, mode)
        errs = [oracle.rel_l2(got[b], oracle.dft(x[b].astype(np.complex128), sign)) for b in range(256)]
        print("dft16 %s sign %d: max rel L2 %.3e" % (mode, sign, max(errs)))
        assert max(errs) <= BOUND[mode], (mode, sign, max(errs))


@pytest.mark.parametrize("mode", ["f16x2", "bf16x2"])
@pytest.mark.parametrize("t,batch", [(4, 64), (8, 8), (12, 4)])
def test_single_pass_transform_error(lf, torch, mode, t, batch):
    """Single-pass plans (whole lines in one workgroup, threads sweeping one
    line first) of 16, 256 and 4096 points on the matrix cores."""
    x = datagen.signals(1 << t, batch, np.complex64, "normal", 162 + t)
    for sign in (-1, 1):
        announce("precision single-pass %s n=2^%d batch=%d sign=%d" % (mode, t, batch, sign))
        plan = lf.Plan(1 << t, batch, torch.complex64)
        assert plan.info()["passes"] == 1
        plan.set_precision(mode)
        xd = to_dev(x)
        y = torch.full_like(xd, float("nan"))
        plan.execute(xd, y, sign)
        torch.cuda.synchronize()
        plan.destroy()
        got = to_np(y)
        ref = oracle.fft_batch(x.astype(np.complex128), sign)
        errs = [oracle.rel_l2(got[b], ref[b]) for b in range(batch)]
        assert max(errs) <= BOUND[mode], (mode, t, sign, errs)


@pytest.mark.parametrize("mode", ["f16x2", "bf16x2"])
@pytest.mark.parametrize("t,batch,log2_p", [(8, 8, 0), (12, 4, 0), (16, 4, 8), (20, 2, 8), (24, 1, 0)])
def test_transform_error(lf, mode, t, batch, log2_p):
    """Whole two-level transforms at 2^8 and 2^12 (the default splits),
    2^16 (256 x 256), 2^20 (4096 x 256) and 2^24 (4096 x 4096)."""
    x = datagen.signals(1 << t, batch, np.complex64, "normal", 62 + t)
    for sign in (-1, 1):
        announce("precision %s n=2^%d batch=%d sign=%d" % (mode, t, batch, sign))
        got = run_prec(lf, x, sign, mode, log2_p=log2_p)
        ref = oracle.fft_batch(x.astype(np.complex128), sign)
        errs = [oracle.rel_l2(got[b], ref[b]) for b in range(batch)]
        print("%s n=2^%d sign %d: max rel L2 %.3e" % (mode, t, sign, max(errs)))
        assert max(errs) <= BOUND[mode], (mode, t, sign, errs)


@pytest.mark.parametrize("mode", ["f16x2", "bf16x2"])
def test_three_level_2p24(lf, torch, mode):
    """The default plan at n = 2^24 (three levels, 256 x 256 x 256, every
    stage radix 16) with its three axis passes on the matrix cores, both
    signs, against the oracle."""
    n = 1 << 24
    x_np = datagen.signals(n, 1, np.complex64, "normal", 64)
    plan = lf.Plan(n, 1, torch.complex64)
    assert plan.info()["levels"] == 3
    plan.set_precision(mode)
    assert plan.info()["precision"] == {"f16x2": 1, "bf16x2": 2}[mode]
    x = to_dev(x_np)
    y = torch.full_like(x, float("nan"))
    for sign in (-1, 1):
        announce("precision three-level n=2^24 %s sign=%d" % (mode, sign))
        plan.execute(x, y, sign)
        torch.cuda.synchronize()
        err = oracle.rel_l2(to_np(y)[0], oracle.fft(x_np[0].astype(np.complex128), sign))
        print("three-level 2^24 %s sign %d: rel L2 %.3e" % (mode, sign, err))
        assert err <= BOUND[mode], (mode, sign, err)
    plan.destroy()


def test_config4_sampled(lf, torch):
    """Config 4: 256 transforms of 2^20, N(0,1) (seed 4), lifted 4096 x 256,
    with FP16 and BF16 pairs: eight sampled transforms against the oracle, and
    every transform finite."""
    n, batch = 1 << 20, 256
    x_np = datagen.signals(n, batch, np.complex64, "normal", 4)
    pick = datagen.sample_indices(batch, 8, seed=4)
    plan = lf.Plan(n, batch, torch.complex64, log2_p=8)
    x = to_dev(x_np)
    y = torch.empty_like(x)
    ref = oracle.fft_batch(x_np[pick].astype(np.complex128), -1)
    for mode in ("f16x2", "bf16x2"):
        announce("precision config4 %s" % mode)
        plan.set_precision(mode)
        plan.execute(x, y, -1)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(torch.view_as_real(y)).all())
        got = to_np(y)
        errs = [oracle.rel_l2(got[b], ref[i]) for i, b in enumerate(pick)]
        print("config4 %s: max rel L2 over 8 sampled transforms %.3e" % (mode, max(errs)))
        assert max(errs) <= BOUND[mode], (mode, errs)
    plan.destroy()


def test_precision_switching_and_errors(lf, torch):
    """Back to FP32 reproduces the FP32 result bit for bit; unsupported shapes
    and types are refused and leave the plan unchanged."""
    n = 1 << 12
    x_np = datagen.signals(n, 4, np.complex64, "normal", 63)
    x = to_dev(x_np)
    plan = lf.Plan(n, 4, torch.complex64)
    y0, y1 = torch.empty_like(x), torch.empty_like(x)
    plan.execute(x, y0, -1)
    plan.set_precision("f16x2")
    plan.execute(x, y1, -1)
    plan.set_precision("fp32")
    plan.execute(x, y1, -1)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(y0).view(np.uint32), to_np(y1).view(np.uint32))
    with pytest.raises(lf.FFTError) as e:
        plan.set_precision(7)
    assert e.value.code == -9
    plan.destroy()
    for make in (lambda: lf.Plan(1 << 22, 1, torch.complex64),            # 2048-point lines
                 lambda: lf.Plan(1 << 25, 1, torch.complex64),            # three levels, 512-point lines
                 lambda: lf.Plan(1 << 12, 1, torch.complex128),           # complex128
                 lambda: lf.Plan(1 << 12, 1, torch.complex64, radix=2),   # radix-2 stages
                 lambda: lf.Plan.uneven([256, 4096], torch.complex64)):   # uneven batch
        p = make()
        with pytest.raises(lf.FFTError) as e:
            p.set_precision("bf16x2")
        assert e.value.code == -8
        assert p.info()["precision"] == 0
        p.destroy()

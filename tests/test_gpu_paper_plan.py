"""The paper's partitioned plan on the GPU (fft_plan_create_paper: Sections
4.2-4.8, Fig. 4.9 -- bit-reversed input, block phase on contiguous blocks,
block-to-cyclic redistribution, cyclic phase with the weightcyclic factors)
against the FP64 oracle, at every valid (m, breakpoint) for n = 2^12 and
2^16, both element types and both signs.

Tolerances as for every other plan: relative L2 per transform 1e-6
(complex64), 1e-12 (complex128).  The radix-2 stage loop has t rounding
levels instead of the lift's three, so its complex64 error is somewhat
larger (still well under 1e-6 at t = 16).
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


def valid_pairs(t):
    """Every (log2 m, breakpoint) of Section 4.8: psize = 2^(t - log2 m) >= m and
    log2 m + 1 <= bp <= log2 psize + 1."""
    return [(lm, bp) for lm in range(0, t // 2 + 1) for bp in range(lm + 1, t - lm + 2)]


@pytest.mark.parametrize("t", [12, 16])
@pytest.mark.parametrize("dt", [np.complex64, np.complex128])
def test_every_breakpoint(lf, torch, t, dt):
    n = 1 << t
    x_np = datagen.signals(n, 1, dt, "normal", 40 + t)
    ref = {s: oracle.fft(x_np[0].astype(np.complex128), s) for s in (-1, 1)}
    tdt = torch.complex64 if dt == np.complex64 else torch.complex128
    x = to_dev(x_np)
    worst = 0.0
    for lm, bp in valid_pairs(t):
        plan = lf.Plan.paper(n, 1, tdt, log2_m=lm, breakpoint=bp)
        info = plan.info()
        assert (info["log2_p"], info["log2_q"], info["paper_breakpoint"]) == (lm, t - lm, bp)
        for sign in (-1, 1):
            announce("paper plan n=2^%d %s log2_m=%d bp=%d sign=%d" % (t, np.dtype(dt).name, lm, bp, sign))
            y = torch.full_like(x, float("nan"))
            plan.execute(x, y, sign)
            torch.cuda.synchronize()
            e = oracle.rel_l2(to_np(y)[0], ref[sign])
            assert e <= TOL[dt], (t, lm, bp, sign, e)
            worst = max(worst, e)
        plan.destroy()
    print("paper plan n=2^%d %s: %d (m, bp) pairs, worst rel L2 %.3g"
          % (t, np.dtype(dt).name, len(valid_pairs(t)), worst))


def test_batch_and_in_place(lf, torch):
    """Batch of 3 at n = 2^14 (m = 8, bp = 6) and an in-place execute."""
    n, batch = 1 << 14, 3
    x_np = datagen.signals(n, batch, np.complex64, "uniform", 47)
    ref = oracle.fft_batch(x_np.astype(np.complex128), -1)
    plan = lf.Plan.paper(n, batch, torch.complex64, log2_m=3, breakpoint=6)
    x = to_dev(x_np)
    y = torch.empty_like(x)
    announce("paper plan batch=3 n=2^14 m=8 bp=6")
    plan.execute(x, y, -1)
    plan.execute(x, x, -1)  # in place: the block phase writes the plan's scratch
    torch.cuda.synchronize()
    for got in (to_np(y), to_np(x)):
        errs = [oracle.rel_l2(got[b], ref[b]) for b in range(batch)]
        assert max(errs) <= 1e-6, errs
    plan.destroy()


def test_private_copies_in_global_memory(lf, torch):
    """psize beyond one workgroup's LDS (2^15 complex64 = 256 KB, 2^14
    complex128) keeps the processors' private copies in global memory."""
    for dt, tdt, lm in ((np.complex64, torch.complex64, 1), (np.complex128, torch.complex128, 2)):
        n = 1 << 16
        x_np = datagen.signals(n, 2, dt, "normal", 48)
        ref = oracle.fft_batch(x_np.astype(np.complex128), 1)
        plan = lf.Plan.paper(n, 2, tdt, log2_m=lm, breakpoint=9)
        assert plan.info()["lds_bytes_pass1"] == 0
        x = to_dev(x_np)
        y = torch.empty_like(x)
        announce("paper plan global private copies %s log2_m=%d" % (np.dtype(dt).name, lm))
        plan.execute(x, y, 1)
        torch.cuda.synchronize()
        got = to_np(y)
        errs = [oracle.rel_l2(got[b], ref[b]) for b in range(2)]
        assert max(errs) <= TOL[dt], errs
        plan.destroy()


def test_argument_checks(lf, torch):
    from paper_0811_2535_amd.binding import FFTError
    for kw in (dict(log2_m=7, breakpoint=8), dict(log2_m=2, breakpoint=2), dict(log2_m=2, breakpoint=12),
               dict(log2_m=-1, breakpoint=1)):
        with pytest.raises(FFTError) as ei:
            lf.Plan.paper(1 << 12, 1, torch.complex64, **kw)
        assert ei.value.name == "FFT_E_ARG", kw
    with pytest.raises(FFTError) as ei:
        lf.Plan.paper(1 << 21, 1, torch.complex64, log2_m=4, breakpoint=6)
    assert ei.value.name == "FFT_E_UNSUPPORTED"

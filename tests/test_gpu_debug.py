"""Debug and failure paths on the device: the NaN-canary mode (scratch and
output filled with quiet NaNs before the passes that write them, so that an
element read before it is written would reach the output as a NaN) and a plan
too large for the device, which must fail with FFT_E_OOM and leave the device's
free memory as it was."""
import numpy as np
import pytest

import datagen
from gpu_util import announce, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

TWO, THREE, CANARY = 128, 256, 4096  # FFT_OPT_TWO_LEVEL, FFT_OPT_THREE_LEVEL, FFT_OPT_DEBUG_CANARY


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lf(torch):
    import paper_0811_2535_amd as lf
    return lf


# single pass, two-level (several splits and tile shapes), three-level, and
# both element types; every case also in place
CASES = [(12, 3, np.complex64, {}), (20, 2, np.complex64, {"flags": TWO}),
         (18, 2, np.complex64, {"flags": TWO, "log2_p": 5}), (24, 1, np.complex64, {"flags": TWO}),
         (22, 1, np.complex64, {"flags": THREE}), (24, 1, np.complex64, {}),
         (16, 2, np.complex128, {"flags": TWO}), (21, 1, np.complex128, {"flags": THREE})]


@pytest.mark.parametrize("t,batch,dtype,opts", CASES)
def test_canary_mode_changes_nothing(lf, torch, t, batch, dtype, opts):
    """With the canary fills the outputs are bit for bit those of the same
    plan without them (so no NaN reached them), out of place and in place,
    for both signs."""
    n = 1 << t
    tdt = torch.complex64 if dtype == np.complex64 else torch.complex128
    x_np = datagen.signals(n, batch, dtype, "normal", 900 + t)
    base = dict(opts)
    flags = base.pop("flags", 0)
    plain = lf.Plan(n, batch, tdt, flags=flags, **base)
    canary = lf.Plan(n, batch, tdt, flags=flags | CANARY, **base)
    assert canary.info()["passes"] == plain.info()["passes"]
    x = to_dev(x_np)
    for sign in (-1, 1):
        announce("canary n=2^%d batch=%d %s opts=%s sign=%d" % (t, batch, np.dtype(dtype).name, opts, sign))
        want = torch.empty_like(x)
        plain.execute(x, want, sign)
        got = torch.zeros_like(x)
        canary.execute(x, got, sign)
        inplace = x.clone()
        canary.execute(inplace, inplace, sign)
        torch.cuda.synchronize()
        w, g, i = to_np(want), to_np(got), to_np(inplace)
        assert not np.isnan(g).any() and not np.isnan(i).any()
        real = np.float32 if dtype == np.complex64 else np.float64
        assert np.array_equal(g.view(real), w.view(real)), (t, opts, sign)
        assert np.array_equal(i.view(real), w.view(real)), (t, opts, sign, "in place")
    plain.destroy()
    canary.destroy()


def test_oversized_plan_fails_with_oom_and_leaks_nothing(lf, torch):
    """A plan whose scratch array (8 TiB) no device memory can hold: every
    attempt returns FFT_E_OOM and the device's free memory is unchanged."""
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(4):
        announce("oversized plan n=2^24 batch=2^16 c64 (expect FFT_E_OOM)")
        with pytest.raises(lf.FFTError) as e:
            lf.Plan(1 << 24, 1 << 16, torch.complex64)
        assert e.value.name == "FFT_E_OOM", e.value
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert abs(free1 - free0) <= (64 << 20), (free0, free1)
    # the library still works afterwards
    x_np = datagen.signals(1 << 16, 1, np.complex64, "normal", 5)
    plan = lf.Plan(1 << 16, 1, torch.complex64)
    x = to_dev(x_np)
    y = torch.empty_like(x)
    plan.execute(x, y, -1)
    torch.cuda.synchronize()
    plan.destroy()
    ref = np.fft.fft(x_np.astype(np.complex128), axis=1)
    assert np.linalg.norm(to_np(y) - ref) <= 1e-6 * np.linalg.norm(ref)

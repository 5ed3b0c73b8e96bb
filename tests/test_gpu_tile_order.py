"""Tile orders (FFT_OPT_TILE_ORDER): the order in which workgroups take their
tiles changes when each tile's memory traffic happens, never what is
computed, so every order must give the same result bit for bit; the library's
measured default orders at n = 2^24 are the ones fft_plan_get_info reports;
orders a launch cannot take are refused."""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import announce, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lf(torch):
    import paper_0811_2535_amd as lf
    return lf


def test_default_orders(lf, torch):
    """The measured default orders of the shapes the library knows
    (complex64, default kernels, FP32); other batches, explicit kernel
    options, FFT_OPT_NO_XCD_REMAP, the matrix-core forms and other lengths
    keep the plain orders (pass B and C of a three-level lift up to 2^24 in
    the hardware order)."""
    B = lf.binding
    cases = [((1 << 24, 1, dict(log2_p=12)), 0x0412),
             ((1 << 24, 1, dict(flags=B.FFT_OPT_TWO_LEVEL)), 0x0412),
             ((1 << 24, 1, {}), 0x800305),
             ((1 << 23, 1, {}), 0x0112),
             ((1 << 25, 1, {}), 0x800005),
             ((1 << 20, 16, {}), 0x8003),
             ((1 << 12, 4096, {}), 0x80),
             ((1 << 24, 2, dict(log2_p=12)), 0x0000),
             ((1 << 24, 1, dict(log2_p=12, flags=B.FFT_OPT_SPLIT_EXCHANGE)), 0x0000),
             ((1 << 24, 1, dict(log2_p=12, lines_per_block=2)), 0x0000),
             ((1 << 24, 1, dict(log2_p=12, flags=B.FFT_OPT_NO_XCD_REMAP)), 0x8080),
             ((1 << 22, 1, {}), 0x0000),
             ((1 << 21, 1, dict(flags=B.FFT_OPT_THREE_LEVEL)), 0x808000)]
    for (n, batch, kw), want in cases:
        announce("tile order default n=%d batch=%d %s" % (n, batch, kw))
        plan = lf.Plan(n, batch, torch.complex64, **kw)
        assert plan.info()["tile_order"] == want, (n, batch, kw, hex(plan.info()["tile_order"]))
        plan.destroy()
    plan = lf.Plan(1 << 24, 1, torch.complex64, log2_p=12)
    plan.set_precision("bf16x2")
    assert plan.info()["tile_order"] == 0x0000
    plan.set_precision("fp32")
    assert plan.info()["tile_order"] == 0x0412
    plan.destroy()


# (n, batch, dtype, options, orders): the first order is the reference
CASES = [
    (1 << 24, 1, np.complex64, dict(log2_p=12), [0x0000, 0x0412, 0x0501, 0x0380, 0x8080, 0x0333]),
    (1 << 24, 1, np.complex64, {}, [0x000000, 0x800305, 0x050505, 0x808080, 0x121212]),
    (1 << 16, 64, np.complex64, {}, [0x0000, 0x0101, 0x1313, 0x8004]),
    (1 << 12, 256, np.complex64, {}, [0x00, 0x02, 0x80, 0x13]),
    (1 << 20, 2, np.complex128, {}, [0x0000, 0x0202, 0x8011]),
    # the other shapes with measured default orders
    (1 << 23, 1, np.complex64, {}, [0x0000, 0x0112]),
    (1 << 25, 1, np.complex64, {}, [0x000000, 0x800005]),
    (1 << 20, 16, np.complex64, {}, [0x0000, 0x8003, 0x0312]),
    (1 << 12, 4096, np.complex64, {}, [0x00, 0x80]),
]


@pytest.mark.parametrize("n,batch,dtype,kw,orders", CASES,
                         ids=["c64-2^24-two-level", "c64-2^24-three-level", "c64-2^16x64",
                              "c64-2^12x256-single", "c128-2^20x2", "c64-2^23", "c64-2^25",
                              "c64-2^20x16", "c64-2^12x4096-single"])
def test_orders_change_no_bit(lf, torch, n, batch, dtype, kw, orders):
    x_np = datagen.signals(n, batch, dtype, "normal", 700 + n.bit_length())
    x = to_dev(x_np)
    tdt = torch.complex64 if dtype == np.complex64 else torch.complex128
    flags = kw.pop("flags", 0) if "flags" in kw else 0
    for sign in (-1, 1):
        ref = None
        for order in orders:
            announce("tile order n=%d batch=%d order=%#x sign=%d" % (n, batch, order, sign))
            # the canary mode fills the scratch array (and `out`) with NaNs before
            # each execute, so a tile that an order skipped cannot be covered up
            # by what an earlier plan left in reused memory
            plan = lf.Plan(n, batch, tdt, flags=flags | lf.binding.FFT_OPT_TILE_ORDER | lf.binding.FFT_OPT_DEBUG_CANARY,
                           tile_order=order, **kw)
            assert plan.info()["tile_order"] == order, hex(plan.info()["tile_order"])
            y = torch.full_like(x, float("nan"))
            plan.execute(x, y, sign)
            torch.cuda.synchronize()
            plan.destroy()
            got = to_np(y)
            if ref is None:
                ref = got
                if n * batch <= 1 << 22:  # the reference order against the oracle
                    want = oracle.fft_batch(x_np.astype(np.complex128), sign)
                    tol = 1e-6 if dtype == np.complex64 else 1e-12
                    errs = [oracle.rel_l2(got[b], want[b]) for b in range(batch)]
                    assert max(errs) <= tol, errs
            else:
                assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), (hex(order), sign)


def test_orders_that_do_not_fit(lf, torch):
    """A spread whose blocks exceed an XCD's range, a spread on a persistent
    pass or on the LDS-staged pass 1: FFT_E_UNSUPPORTED; a byte for a pass
    the plan does not have: FFT_E_ARG."""
    B = lf.binding
    cases = [((1 << 24, dict(log2_p=12, tile_order=0x000f)), -8),   # 2^15 tiles per run > 256
             ((1 << 24, dict(log2_p=12, tile_order=0x7700)), -8),   # 2^14 > 128
             ((1 << 24, dict(log2_p=12, tile_order=0x02, flags=B.FFT_OPT_PERSISTENT)), -8),
             ((1 << 24, dict(log2_p=12, tile_order=0x02, flags=B.FFT_OPT_TWO_LEVEL | B.FFT_OPT_LDS_PREFETCH)), -8),
             ((1 << 12, dict(tile_order=0x0100)), -9),               # single pass
             ((1 << 20, dict(tile_order=0x010000)), -9)]             # two passes
    for (n, kw), code in cases:
        kw = dict(kw)
        kw["flags"] = kw.get("flags", 0) | B.FFT_OPT_TILE_ORDER
        announce("tile order refused n=%d %s" % (n, kw))
        with pytest.raises(lf.FFTError) as e:
            lf.Plan(n, 1, torch.complex64, **kw)
        assert e.value.code == code, (n, kw, e.value.code)

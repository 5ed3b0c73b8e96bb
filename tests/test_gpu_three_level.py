"""Three-level lift n = n1 n2 n3 (three axis passes) against the FP64 oracle,
through the C ABI.

Same tolerances as the two-level path: relative L2 per transform <= 1e-6
(complex64), 1e-12 (complex128), against the oracle run on exactly the values
the GPU received.  Sizes span every factorisation the plan makes from
2^15 = 32^3 up to 2^24 = 256^3 (full oracle), batches with more than one
transform, both signs, in-place execution, and 2^25..2^28 complex64 (full
oracle at 2^25/2^26 and complex128 2^27; tone, round trip and sampled
frequencies at 2^28 and at the largest lengths, 2^30 complex64 and 2^29
complex128).
"""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import announce, require_gpu, to_dev, to_np

TOL = {np.complex64: 1e-6, np.complex128: 1e-12}
pytestmark = pytest.mark.gpu
THREE = 256  # FFT_OPT_THREE_LEVEL
TWO = 128    # FFT_OPT_TWO_LEVEL


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def lf(torch):
    import paper_0811_2535_amd as lf
    return lf


def factors(t):
    l3 = (t + 2) // 3
    l1 = (t - l3 + 1) // 2
    return l1, t - l3 - l1, l3


def run3(lf, x_np, sign, flags=THREE, in_place=False, **opts):
    import torch
    batch, n = x_np.shape
    dt = torch.complex64 if x_np.dtype == np.complex64 else torch.complex128
    plan = lf.Plan(n, batch, dt, flags=flags, **opts)
    info = plan.info()
    x = to_dev(x_np)
    if in_place:
        plan.execute(x, x, sign)
        y = x
    else:
        y = torch.full_like(x, float("nan"))
        plan.execute(x, y, sign)
    torch.cuda.synchronize()
    plan.destroy()
    return to_np(y), info


def dft_at(x, k, sign):
    """X_k = sum_j x_j exp(sign 2 pi i (j k mod n) / n) in FP64, in chunks."""
    n = x.size
    acc = 0j
    step = 1 << 22
    for j0 in range(0, n, step):
        j = np.arange(j0, min(n, j0 + step), dtype=np.int64)
        e = (j * np.int64(k)) % n
        acc += np.sum(x[j0:j0 + j.size].astype(np.complex128) * np.exp(sign * 2j * np.pi * (e / n)))
    return acc


def check(got, x_np, sign, tol, what):
    ref = oracle.fft_batch(x_np.astype(np.complex128), sign)
    assert not np.isnan(got).any(), (what, "NaN left in the output")
    errs = [oracle.rel_l2(got[b], ref[b]) for b in range(x_np.shape[0])]
    assert max(errs) <= tol, (what, errs)
    return max(errs)


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128], ids=["c64", "c128"])
@pytest.mark.parametrize("t", list(range(15, 23)))
def test_every_factorisation(lf, t, dtype):
    batch = 3 if t <= 20 else 1
    x = datagen.signals(1 << t, batch, dtype, "normal", 900 + t)
    for sign in (-1, 1):
        announce("three-level n=2^%d %s batch=%d sign=%d" % (t, np.dtype(dtype).name, batch, sign))
        got, info = run3(lf, x, sign)
        l1, l2, l3 = factors(t)
        assert info["passes"] == 3 and info["levels"] == 3
        assert (info["log2_n1"], info["log2_n2"], info["log2_n3"]) == (l1, l2, l3)
        check(got, x, sign, TOL[dtype], (t, sign))


def test_full_size_2p24(lf, torch):
    """n = 2^24 = 256^3 complex64, N(0,1) seed 2: forward and inverse against
    the full oracle, and the round trip."""
    n = 1 << 24
    x_np = datagen.signals(n, 1, np.complex64, "normal", 2)
    plan = lf.Plan(n, 1, torch.complex64, flags=THREE)
    info = plan.info()
    assert (info["log2_n1"], info["log2_n2"], info["log2_n3"]) == (8, 8, 8)
    # each pass reads and writes rows of at least 128 contiguous bytes
    for k in (1, 2, 3):
        assert info["lines_per_block_pass%d" % k] * 8 >= 128
    x = to_dev(x_np)
    y, z, w = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
    announce("three-level n=2^24 forward + inverse of forward + inverse")
    plan.execute(x, y, -1)
    plan.execute(y, z, 1)
    plan.execute(x, w, 1)
    torch.cuda.synchronize()
    plan.destroy()
    e_f = oracle.rel_l2(to_np(y)[0], oracle.fft(x_np[0].astype(np.complex128), -1))
    e_i = oracle.rel_l2(to_np(w)[0], oracle.fft(x_np[0].astype(np.complex128), 1))
    e_rt = oracle.rel_l2(to_np(z)[0] / n, x_np[0])
    assert e_f <= 1e-6 and e_i <= 1e-6 and e_rt <= 2e-6, (e_f, e_i, e_rt)


@pytest.mark.parametrize("t,dtype", [(18, np.complex64), (21, np.complex128)])
def test_in_place_and_batch(lf, t, dtype):
    x = datagen.signals(1 << t, 4, dtype, "uniform", 950 + t)
    announce("three-level in place n=2^%d batch=4" % t)
    got, _ = run3(lf, x, -1, in_place=True)
    check(got, x, -1, TOL[dtype], ("in place", t))


def test_agrees_with_two_level(lf):
    """Both lifts of the same transform agree to rounding level."""
    t = 22
    x = datagen.signals(1 << t, 2, np.complex64, "normal", 960)
    announce("three-level vs two-level n=2^22")
    a, _ = run3(lf, x, -1)
    b, info2 = run3(lf, x, -1, flags=TWO)
    assert info2["passes"] == 2
    scale = np.abs(b).max()
    assert np.abs(a.astype(np.complex128) - b).max() <= 1e-5 * scale


@pytest.mark.parametrize("T", [16, 32, 64])
def test_tile_widths_and_split_exchange(lf, T):
    t = 21
    x = datagen.signals(1 << t, 2, np.complex64, "normal", 970)
    for flags in (THREE, THREE | 2):
        announce("three-level T=%d flags=%d" % (T, flags))
        got, info = run3(lf, x, 1, flags=flags, lines_per_block=T)
        assert info["lines_per_block_pass1"] == T and info["lines_per_block_pass3"] == T
        assert info["variant_pass1"] == (2 if flags & 2 else 0)
        check(got, x, 1, 1e-6, (T, flags))


@pytest.mark.parametrize("t", [25, 26])
def test_full_oracle_beyond_2p24(lf, torch, t):
    n = 1 << t
    x_np = datagen.signals(n, 1, np.complex64, "normal", 980 + t)
    announce("three-level n=2^%d forward" % t)
    got, info = run3(lf, x_np, -1)
    assert info["levels"] == 3
    err = oracle.rel_l2(got[0], oracle.fft(x_np[0].astype(np.complex128), -1))
    assert err <= 1e-6, err


@pytest.mark.parametrize("t,dtype", [(28, np.complex64), (30, np.complex64), (29, np.complex128)],
                         ids=["c64-28", "c64-30", "c128-29"])
def test_properties_at_limit(lf, torch, t, dtype):
    """The largest lengths: 2^28 complex64 (the last addressed with 32-bit
    buffer offsets) and 2^30 complex64 / 2^29 complex128 (8 GiB per buffer,
    addressed in 64 bits): a pure tone lands in its bin, the round trip
    returns n x, and sampled outputs match the FP64 sum."""
    n = 1 << t
    tdt = torch.complex64 if dtype == np.complex64 else torch.complex128
    tol = 1e-6 if dtype == np.complex64 else 1e-12
    plan = lf.Plan(n, 1, tdt, flags=THREE)
    assert plan.info()["levels"] == 3
    a = 98765 % n
    j = torch.arange(n, device="cuda", dtype=torch.int64)
    ang = (j * a % n).to(torch.float64) * (2 * np.pi / n)
    del j
    x = torch.complex(torch.cos(ang), torch.sin(ang)).to(tdt)
    del ang
    y = torch.empty_like(x)
    announce("three-level limit n=2^%d %s tone" % (t, np.dtype(dtype).name))
    plan.execute(x, y, -1)
    torch.cuda.synchronize()
    y[a] -= n
    err = float(torch.linalg.vector_norm(y.to(torch.complex128)) / n)
    assert err <= tol, err
    del x
    torch.cuda.empty_cache()
    x_np = datagen.signals(n, 1, dtype, "normal", 990 + t)[0]
    x = to_dev(x_np)
    announce("three-level limit n=2^%d %s round trip" % (t, np.dtype(dtype).name))
    plan.execute(x, y, -1)
    z = torch.empty_like(y)
    plan.execute(y, z, 1)
    torch.cuda.synchronize()
    rt = float(torch.linalg.vector_norm((z / n - x).to(torch.complex128)) /
               torch.linalg.vector_norm(x.to(torch.complex128)))
    assert rt <= 2 * tol, rt
    del z
    y_np = to_np(y)
    plan.destroy()
    rms = np.sqrt(np.mean(np.abs(y_np.astype(np.complex128)) ** 2))
    for k in datagen.sample_indices(n, 3 if t <= 28 else 1, seed=t):
        announce("three-level limit n=2^%d sample k=%d" % (t, k))
        ref = dft_at(x_np, int(k), -1)
        assert abs(y_np[k] - ref) <= 10 * tol * rms, (k, y_np[k], ref)


def test_full_oracle_c128_2p27(lf, torch):
    """The largest complex128 length still addressed with buffer descriptors,
    against the full oracle."""
    t = 27
    x_np = datagen.signals(1 << t, 1, np.complex128, "normal", 1027)
    announce("three-level n=2^27 c128 forward")
    got, info = run3(lf, x_np, -1)
    assert info["levels"] == 3
    err = oracle.rel_l2(got[0], oracle.fft(x_np[0], -1))
    assert err <= 1e-12, err


def test_timing_precision_and_errors(lf, torch):
    n = 1 << 20
    plan = lf.Plan(n, 1, torch.complex64, flags=THREE)
    x = torch.zeros(n, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    plan.set_timing(True)
    for _ in range(3):
        plan.execute(x, y, -1)
    ms, cnt = plan.read_timing()
    plan.set_timing(False)
    assert cnt == [3, 3, 3] and min(ms) > 0
    plan.set_precision("fp32")
    with pytest.raises(lf.FFTError) as e:
        plan.set_precision("f16x2")  # 2^20 = 128 x 64 x 128: lines not all radix 16
    assert e.value.code == -8
    plan.destroy()
    for t, opts, code in ((14, {}, -8), (20, dict(radix=2), -8), (20, dict(lines_per_block=3), -9),
                          (20, dict(lines_per_block=256), -8), (20, dict(values_per_thread=32), -8),
                          (20, dict(flags=THREE | 8), -8)):
        with pytest.raises(lf.FFTError) as e:
            lf.Plan(1 << t, 1, torch.complex64, **dict(dict(flags=THREE), **opts))
        assert e.value.code == code, (t, opts)


def test_default_lift_by_size(lf, torch):
    """The library lifts to three levels from 2^24 on (both element types)
    unless a two-level option is given, and to two levels below."""
    cases = [(23, torch.complex64, {}, 2), (24, torch.complex64, {}, 3), (24, torch.complex128, {}, 3),
             (24, torch.complex64, dict(flags=TWO), 2), (24, torch.complex64, dict(log2_p=12), 2),
             (24, torch.complex64, dict(lines_per_block=2), 2), (24, torch.complex64, dict(flags=2), 2),
             (24, torch.complex64, dict(radix=2), 2), (22, torch.complex64, dict(flags=THREE), 3)]
    for t, dt, opts, levels in cases:
        p = lf.Plan(1 << t, 1, dt, **opts)
        info = p.info()
        p.destroy()
        assert info["levels"] == info["passes"] == levels, (t, dt, opts, info["levels"])



SHUFFLE = 512  # FFT_OPT_SHUFFLE_EXCHANGE


@pytest.mark.parametrize("t,batch", [(24, 1), (23, 1), (22, 2), (25, 1)])
def test_shuffle_exchange(lf, torch, t, batch):
    """Axis passes over 256-point lines with the stage exchange done by
    wavefront shuffles (DPP and ds_swizzle within 16-lane rows); passes over
    other lengths keep the LDS-tile kernel.  Both signs, against the oracle,
    and in place."""
    n = 1 << t
    x_np = datagen.signals(n, batch, np.complex64, "normal", 90 + t)
    l1, l2, l3 = factors(t)
    for sign in (-1, 1):
        announce("three-level shuffle exchange t=%d batch=%d sign=%d" % (t, batch, sign))
        got, info = run3(lf, x_np, sign, flags=THREE | SHUFFLE)
        shuffled = [bool(info[k] & 64) for k in ("variant_pass1", "variant_pass2")]
        assert shuffled == [l3 == 8, l2 == 8], (t, info)
        check(got, x_np, sign, 1e-6, "shuffle t=%d" % t)
    got, _ = run3(lf, x_np, -1, flags=THREE | SHUFFLE, in_place=True)
    check(got, x_np, -1, 1e-6, "shuffle in place t=%d" % t)


def test_shuffle_exchange_refusals(lf, torch):
    from paper_0811_2535_amd.binding import FFTError
    for n, dt, flags, want in ((1 << 24, torch.complex128, THREE | SHUFFLE, "FFT_E_UNSUPPORTED"),
                               (1 << 18, torch.complex64, THREE | SHUFFLE, "FFT_E_UNSUPPORTED"),
                               (1 << 24, torch.complex64, SHUFFLE, "FFT_E_ARG"),
                               (1 << 24, torch.complex64, THREE | SHUFFLE | 2, "FFT_E_ARG")):
        with pytest.raises(FFTError) as ei:
            lf.Plan(n, 1, dt, flags=flags)
        assert ei.value.name == want, (n, dt, flags)

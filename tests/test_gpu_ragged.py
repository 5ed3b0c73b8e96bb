"""Packed batches of uneven power-of-two lengths (fft_plan_create_many)
against the FP64 oracle, transform by transform, through the C ABI.

The oracle runs on exactly the values the GPU received; transforms of equal
length are handed to it as one batch.  Tolerances as for single-length plans:
relative L2 per transform <= 1e-6 (complex64), 1e-12 (complex128).
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


def oracle_ragged(x, lengths, sign):
    """FP64 oracle of every transform of a packed batch (batched by length)."""
    x = x.astype(np.complex128)
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    out = np.empty_like(x)
    for ln in sorted(set(int(v) for v in lengths)):
        idx = [i for i, v in enumerate(lengths) if v == ln]
        block = np.stack([x[offs[i]:offs[i] + ln] for i in idx])
        ref = oracle.fft_batch(block, sign)
        for k, i in enumerate(idx):
            out[offs[i]:offs[i] + ln] = ref[k]
    return out


def run_ragged(lf, x_np, lengths, sign, graph=False, repeat=1, persistent=False, autotune=False):
    import torch
    dt = torch.complex64 if x_np.dtype == np.complex64 else torch.complex128
    plan = lf.Plan.uneven(lengths, dt, graph=graph, persistent=persistent, autotune=autotune)
    x = to_dev(x_np)
    outs = []
    for _ in range(repeat):
        y = torch.full_like(x, float("nan"))
        plan.execute(x, y, sign)
        torch.cuda.synchronize()
        outs.append(to_np(y))
    info = plan.info()
    plan.destroy()
    return (outs[0] if repeat == 1 else outs), info


def check_ragged(got, ref, lengths, tol, what):
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    assert not np.isnan(got).any(), (what, "NaN left in the output")
    errs = [oracle.rel_l2(got[o:o + ln], ref[o:o + ln]) for o, ln in zip(offs, lengths)]
    worst = int(np.argmax(errs))
    assert max(errs) <= tol, (what, max(errs), "transform", worst, "length", lengths[worst])
    return max(errs)


FORMS = [False, True]  # class plans on forked streams (default); persistent launches
FORM_IDS = ["classes", "persistent"]


@pytest.mark.parametrize("persistent", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128], ids=["c64", "c128"])
def test_every_length_class(lf, dtype, persistent):
    """Every length 2^1..2^16 (single-pass classes up to 2^14 complex64 /
    2^13 complex128, lifted ones above) in one packed batch with random extra
    lengths, both signs."""
    ks = list(datagen.uneven_log2_lengths(160, 1, 16, seed=31)) + list(range(1, 17))
    lengths = [1 << int(k) for k in ks]
    x = datagen.ragged_signals(lengths, dtype, "uniform", 32)
    for sign in (-1, 1):
        announce("ragged every-class %s sign=%d count=%d persistent=%d"
                 % (np.dtype(dtype).name, sign, len(lengths), persistent))
        got, info = run_ragged(lf, x, lengths, sign, persistent=persistent)
        assert info["length_classes"] == 16 and info["passes"] == 2
        assert info["streams"] == (0 if persistent else 4)
        check_ragged(got, oracle_ragged(x, lengths, sign), lengths, TOL[dtype], ("classes", sign))


@pytest.mark.parametrize("persistent", FORMS, ids=FORM_IDS)
def test_config3_full(lf, persistent):
    """4096 transforms with k ~ U{8..16} (seed 3), complex64, U[-1,1]: the
    whole batch against the oracle, forward and inverse."""
    ks = datagen.uneven_log2_lengths(4096, 8, 16, seed=3)
    lengths = [1 << int(k) for k in ks]
    x = datagen.ragged_signals(lengths, np.complex64, "uniform", 3)
    for sign in (-1, 1):
        announce("ragged config3 sign=%d elements=%d persistent=%d" % (sign, len(x), persistent))
        got, info = run_ragged(lf, x, lengths, sign, persistent=persistent)
        assert info["length_classes"] == 9 and info["graph_launch"] == 0
        check_ragged(got, oracle_ragged(x, lengths, sign), lengths, 1e-6, ("config3", sign))


@pytest.mark.parametrize("persistent", FORMS, ids=FORM_IDS)
def test_long_transforms_in_batch(lf, persistent):
    """Lifted lengths up to 2^24 (the three-level lift in the class form)
    mixed with short ones, and a batch whose only length is lifted (no
    single-pass class)."""
    for lengths in ([1 << 22, 256, 1 << 13, 2, 1 << 20, 1 << 13], [1 << 18, 1 << 18],
                    [1 << 24, 1 << 10, 1 << 16]):
        x = datagen.ragged_signals(lengths, np.complex64, "normal", 41)
        announce("ragged long %s persistent=%d" % (lengths, persistent))
        got, _ = run_ragged(lf, x, lengths, -1, persistent=persistent)
        check_ragged(got, oracle_ragged(x, lengths, -1), lengths, 1e-6, lengths)


def test_only_short_transforms(lf):
    lengths = [2, 4, 8, 16, 4096, 4096, 1024, 2] * 7
    x = datagen.ragged_signals(lengths, np.complex128, "uniform", 42)
    announce("ragged short-only c128")
    got, info = run_ragged(lf, x, lengths, 1)
    assert info["passes"] == 1 and info["grid_pass2"] == 0
    check_ragged(got, oracle_ragged(x, lengths, 1), lengths, 1e-12, "short")


@pytest.mark.parametrize("persistent", FORMS, ids=FORM_IDS)
def test_graph_replays_match_direct_launches(lf, torch, persistent):
    """Graph replays (several, with eager work and synchronisations between
    them) give exactly the result of direct launches, for both signs and two
    buffer pairs; in the class form the graph holds the classes' streams as
    parallel branches."""
    ks = datagen.uneven_log2_lengths(300, 4, 15, seed=43)
    lengths = [1 << int(k) for k in ks]
    x_np = datagen.ragged_signals(lengths, np.complex64, "uniform", 43)
    direct = {s: run_ragged(lf, x_np, lengths, s, graph=False, persistent=persistent)[0] for s in (-1, 1)}
    plan = lf.Plan.uneven(lengths, torch.complex64, graph=True, persistent=persistent)
    xs = [to_dev(x_np), to_dev(x_np)]
    ys = [torch.empty_like(xs[0]), torch.empty_like(xs[0])]
    for rep in range(4):
        for s in (-1, 1):
            for b in range(2):
                announce("ragged graph replay rep=%d sign=%d buf=%d" % (rep, s, b))
                ys[b].fill_(float("nan"))
                scratch = torch.randn(1 << 16, device=xs[0].device)  # eager work between replays
                (scratch * 2).sum().item()
                plan.execute(xs[b], ys[b], s)
                torch.cuda.synchronize()
                got = to_np(ys[b])
                assert np.array_equal(got.view(np.uint32), direct[s].view(np.uint32)), (rep, s, b)
    info = plan.info()
    plan.destroy()
    assert info["graph_launch"] == 1


def test_in_place_and_single_length_agreement(lf, torch):
    """In-place execution, and agreement with single-length plans of the same
    transforms to rounding level."""
    lengths = [1 << 14, 512, 1 << 16, 4096, 64, 1 << 14, 512]
    x_np = datagen.ragged_signals(lengths, np.complex64, "normal", 44)
    plan = lf.Plan.uneven(lengths, torch.complex64)
    x = to_dev(x_np)
    announce("ragged in place")
    plan.execute(x, x, -1)
    torch.cuda.synchronize()
    got = to_np(x)
    plan.destroy()
    ref = oracle_ragged(x_np, lengths, -1)
    check_ragged(got, ref, lengths, 1e-6, "in place")
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    for o, ln in zip(offs, lengths):
        single = lf.fft(to_dev(x_np[o:o + ln]), -1)
        s = to_np(single)
        scale = np.abs(s).max()
        assert np.abs(got[o:o + ln].astype(np.complex128) - s).max() <= 1e-5 * scale, ln


def test_ragged_timing_and_errors(lf, torch):
    lengths = [256, 1 << 13, 1024]
    plan = lf.Plan.uneven(lengths, torch.complex64)
    x = torch.zeros(sum(lengths), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    plan.set_timing(True)
    for _ in range(3):
        plan.execute(x, y, -1)
    ms, cnt = plan.read_timing()
    plan.set_timing(False)
    assert cnt[0] == 3 and ms[0] > 0
    with pytest.raises(lf.FFTError):
        plan.execute(x[:-1], y[:-1], -1)
    with pytest.raises(lf.FFTError):
        plan.execute(x, y, 0)
    plan.destroy()


def test_autotuned_classes(lf, torch):
    """FFT_OPT_AUTOTUNE: every class shaped by the tuner (16 candidates per
    shape), both signs, against the oracle."""
    lengths = [1 << 16] * 3 + [1 << 10] * 20 + [1 << 19] * 2 + [64] * 9
    x = datagen.ragged_signals(lengths, np.complex64, "normal", 45)
    for sign in (-1, 1):
        announce("ragged autotuned classes sign=%d" % sign)
        got, info = run_ragged(lf, x, lengths, sign, autotune=True)
        assert info["length_classes"] == 4
        check_ragged(got, oracle_ragged(x, lengths, sign), lengths, 1e-6, ("autotune", sign))

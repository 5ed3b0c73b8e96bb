"""Autotuned plans: the chosen configuration is at least as fast as the
default one (by the tuner's own timing), computes the transform to the usual
tolerance against the FP64 oracle, and is remembered for the shape."""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import announce, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.mark.parametrize("t,batch,dtype,tol,cands", [(20, 2, np.complex64, 1e-6, 16),
                                                      (10, 3, np.complex128, 1e-12, 8),
                                                      (24, 1, np.complex64, 1e-6, 24)])
def test_tuned_plan(torch, t, batch, dtype, tol, cands):
    import paper_0811_2535_amd as lf
    n = 1 << t
    tdt = torch.complex64 if dtype == np.complex64 else torch.complex128
    announce("tune n=2^%d batch=%d %s candidates=%d" % (t, batch, np.dtype(dtype).name, cands))
    plan, res = lf.Plan.tuned(n, batch, tdt, max_candidates=cands)
    # max_candidates bounds the first stage; the tile-order stage adds at most 5 per pass
    assert 2 <= res["candidates"] <= cands + 5 * plan.info()["levels"], res
    assert 0 < res["ms"] <= res["ms_default"], res
    x_np = datagen.signals(n, batch, dtype, "normal", 500 + t)
    x = to_dev(x_np)
    for sign in (-1, 1):
        y = torch.full_like(x, float("nan"))
        plan.execute(x, y, sign)
        torch.cuda.synchronize()
        got = to_np(y)
        ref = oracle.fft_batch(x_np.astype(np.complex128), sign)
        errs = [oracle.rel_l2(got[b], ref[b]) for b in range(batch)]
        assert max(errs) <= tol, (res, sign, errs)
    plan.destroy()
    # the same shape again: the remembered configuration, no new timing
    plan2, res2 = lf.Plan.tuned(n, batch, tdt, max_candidates=cands)
    assert res2 == res
    plan2.destroy()


CACHE_CHILD = r"""
import json, os, sys
sys.path.insert(0, sys.argv[1])
import torch
import paper_0811_2535_amd as lf
plan, res = lf.Plan.tuned(int(sys.argv[2]), int(sys.argv[3]), torch.complex64, max_candidates=4)
info = plan.info()
plan.destroy()
print(json.dumps({"res": res, "info": {k: info[k] for k in ("passes", "log2_p")}}))
"""


def test_tuner_cache_file(torch, tmp_path):
    """With LIFTFFT_TUNE_CACHE set, a tuning outcome is appended to the file
    as one JSON line keyed by (arch, n, batch, dtype), and a fresh process
    asking for the same shape returns the stored configuration and timings
    without tuning (the last matching line wins)."""
    import json
    import os
    import subprocess
    import sys

    import paper_0811_2535_amd as lf
    path = tmp_path / "tune.jsonl"
    n, batch = 1 << 14, 5  # a shape no other test tunes in this process
    os.environ["LIFTFFT_TUNE_CACHE"] = str(path)
    try:
        announce("tune cache: tune n=2^14 batch=5 into %s" % path)
        plan, res = lf.Plan.tuned(n, batch, torch.complex64, max_candidates=4)
        plan.destroy()
    finally:
        del os.environ["LIFTFFT_TUNE_CACHE"]
    lines = path.read_text().splitlines()
    assert len(lines) == 1, lines
    rec = json.loads(lines[0])
    assert rec["arch"].startswith("gfx950"), rec
    assert (rec["n"], rec["batch"], rec["dtype"]) == (n, batch, 0), rec
    assert rec["candidates"] == res["candidates"] and abs(rec["ms"] - res["ms"]) <= 1e-6 * max(1.0, res["ms"])
    # a later line for the same key, naming a configuration the tuner would
    # not report by itself: the two-level lift 64 x 256
    # (every option field is set: the tuner's own line may carry a tile order,
    # which without FFT_OPT_TILE_ORDER in flags would make the line invalid)
    forged = dict(rec, log2_p=6, radix=0, lines_per_block=0, lines_per_block2=0, flags=128, values_per_thread=0,
                  values_per_thread2=0, scratch_width=0, tile_order=0, ms=123.0, ms_default=456.0, candidates=99)
    with open(path, "a") as f:
        f.write(json.dumps(forged) + "\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, LIFTFFT_TUNE_CACHE=str(path))
    announce("tune cache: fresh process reads n=2^14 batch=5 from the file")
    out = subprocess.run([sys.executable, "-c", CACHE_CHILD, root, str(n), str(batch)], env=env,
                         capture_output=True, text=True, timeout=180)
    assert out.returncode == 0, out.stderr[-2000:]
    got = json.loads(out.stdout.strip().splitlines()[-1])
    assert got["res"]["ms"] == 123.0 and got["res"]["candidates"] == 99, got
    assert got["res"]["opts"]["log2_p"] == 6 and got["res"]["opts"]["flags"] == 128, got
    assert got["info"]["passes"] == 2 and got["info"]["log2_p"] == 6, got
    assert len(path.read_text().splitlines()) == 2  # a hit appends nothing

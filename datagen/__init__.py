"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds random-number plumbing only and none of the transform's
arithmetic, so that the GPU path and the FP64 oracle can be fed the same
values without sharing any code with each other.

Recipe (one stream per transform): ``numpy.random.default_rng`` over
``SeedSequence(seed).spawn(batch)[b]``; real and imaginary parts are drawn in
FP64 (``"normal"``: iid standard normal, ``"uniform"``: iid uniform[-1, 1])
and then rounded once to the requested complex dtype.  The oracle receives
exactly those rounded values upcast to complex128.
"""
from __future__ import annotations

import numpy as np

DISTS = ("normal", "uniform")


def _draw(rng: np.random.Generator, n: int, dist: str) -> np.ndarray:
    if dist == "normal":
        re = rng.standard_normal(n)
        im = rng.standard_normal(n)
    elif dist == "uniform":
        re = rng.uniform(-1.0, 1.0, n)
        im = rng.uniform(-1.0, 1.0, n)
    else:
        raise ValueError("unknown distribution %r (expected one of %s)" % (dist, DISTS))
    out = np.empty(n, dtype=np.complex128)
    out.real = re
    out.imag = im
    return out


def signals(n: int, batch: int = 1, dtype=np.complex64, dist: str = "normal",
            seed: int = 0) -> np.ndarray:
    """``(batch, n)`` array of seeded complex signals rounded to ``dtype``."""
    if n < 0 or batch < 0:
        raise ValueError("n and batch must be non-negative")
    streams = np.random.SeedSequence(seed).spawn(batch)
    out = np.empty((batch, n), dtype=dtype)
    for b, ss in enumerate(streams):
        out[b] = _draw(np.random.default_rng(ss), n, dist).astype(dtype)
    return out


def real_weights(n: int, batch: int = 1, seed: int = 0) -> np.ndarray:
    """``(batch, n)`` float64 weights iid uniform[0, 1] (the loss weights w)."""
    streams = np.random.SeedSequence([seed, 0x77]).spawn(batch)
    return np.stack([np.random.default_rng(ss).uniform(0.0, 1.0, n) for ss in streams]) \
        if batch else np.empty((0, n))


def uneven_log2_lengths(count: int, lo: int, hi: int, seed: int = 0) -> np.ndarray:
    """``count`` exponents k drawn uniformly from ``lo..hi`` inclusive."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x3c]))
    return rng.integers(lo, hi + 1, size=count).astype(np.int64)


def ragged_signals(lengths, dtype=np.complex64, dist: str = "uniform",
                   seed: int = 0) -> np.ndarray:
    """Concatenation of one seeded signal per entry of ``lengths``."""
    lengths = [int(v) for v in lengths]
    streams = np.random.SeedSequence(seed).spawn(len(lengths))
    out = np.empty(sum(lengths), dtype=dtype)
    off = 0
    for ln, ss in zip(lengths, streams):
        out[off:off + ln] = _draw(np.random.default_rng(ss), ln, dist).astype(dtype)
        off += ln
    return out


def sample_indices(n: int, count: int, seed: int = 0) -> np.ndarray:
    """``count`` distinct sorted indices in ``[0, n)`` (for sampled checks)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5a]))
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)

"""The paper's staged radix-2 FFT and its block/cyclic parallel plan, restated
in numpy for tests.

Written from the paper's prose description (Sections 2-4), not from its
printed loop nests: this is an independent, iterative formulation of the same
transform, used to pin the recursive FP64 oracle and to fix the readings of
the paper (sign of the weights, breakpoint range, ownership sets).

* :func:`bit_reverse_perm` -- the permutation P_n of Fig. 2.1 (line 1).
* :func:`staged_fft` -- Fig. 2.1 as an in-place stage loop: after P_n, stage
  q = 1..t views x as columns of length L = 2^q (column-major reshape,
  Section 3.3) and replaces each column by B_L times it, i.e. the butterfly of
  Section 3.5 (c = weight * lower half; upper <- upper + c; lower <- upper - c).
* :func:`partitioned_fft` -- the plan of Section 4 with ``m`` virtual
  processors: stages 1..breakpoint-1 run per processor on its private copy of
  the ``psize = n/m`` contiguous elements it owns (the "block" phase,
  Section 4.2 / 4.7); the data is then redistributed so that processor p owns
  the elements whose index is congruent to p mod m (the "cyclic" phase,
  Section 4.3 / 4.6) and stages breakpoint..t run on that private copy using
  only the weights it needs (Sections 4.4 / 4.5).  Valid for
  log2(m)+1 <= breakpoint <= log2(psize)+1 (Section 4.8).
"""
from __future__ import annotations

import numpy as np


def bit_reverse_perm(n: int) -> np.ndarray:
    """Index array ``perm`` with ``perm[i]`` = i with its log2(n) bits reversed."""
    t = n.bit_length() - 1
    if n < 1 or (1 << t) != n:
        raise ValueError("n must be a power of two")
    idx = np.arange(n, dtype=np.int64)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(t):
        rev |= ((idx >> b) & 1) << (t - 1 - b)
    return rev


def _weights(rows: np.ndarray, L: int, sign: int) -> np.ndarray:
    # w_L^(sign*row), each computed directly from its integer exponent.
    ang = 2.0 * np.pi * rows.astype(np.float64) / L
    return np.cos(ang) + 1j * sign * np.sin(ang)


def _stage_on_columns(cols: np.ndarray, w: np.ndarray) -> None:
    """B_L applied to every row of ``cols`` (each row is one column of length
    L in the paper's column-major picture); ``w`` holds the L/2 weights."""
    h = cols.shape[1] // 2
    upper = cols[:, :h].copy()
    c = cols[:, h:] * w
    cols[:, :h] = upper + c
    cols[:, h:] = upper - c


def staged_fft(x, sign: int = 1) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    n = x.size
    t = n.bit_length() - 1
    y = x[bit_reverse_perm(n)].copy()
    for q in range(1, t + 1):
        L = 1 << q
        _stage_on_columns(y.reshape(n // L, L), _weights(np.arange(L // 2), L, sign))
    return y


def breakpoint_range(n: int, m: int) -> tuple[int, int]:
    """Inclusive range of valid breakpoints for m processors (Section 4.8)."""
    psize = n // m
    return (m.bit_length() - 1) + 1, (psize.bit_length() - 1) + 1


def partitioned_fft(x, m: int, breakpoint: int, sign: int = 1,
                    trace: dict | None = None) -> np.ndarray:
    """Section 4's plan with m virtual processors (run one after another).

    If ``trace`` is a dict it receives, per processor, the global indices each
    phase owned ("block", "cyclic"), so tests can check the ownership sets and
    their disjointness."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.size
    t = n.bit_length() - 1
    if m < 1 or n % m or m & (m - 1):
        raise ValueError("m must be a power of two dividing n")
    psize = n // m
    if psize < m:
        raise ValueError("the plan assumes psize >= m")
    lo, hi = breakpoint_range(n, m)
    if not lo <= breakpoint <= hi:
        raise ValueError("breakpoint %d outside [%d, %d]" % (breakpoint, lo, hi))
    y = x[bit_reverse_perm(n)].copy()

    # Block phase: processor p privately owns y[p*psize : (p+1)*psize].
    for p in range(m):
        own = np.arange(p * psize, (p + 1) * psize)
        priv = y[own].copy()
        for q in range(1, breakpoint):
            L = 1 << q
            _stage_on_columns(priv.reshape(psize // L, L),
                              _weights(np.arange(L // 2), L, sign))
        y[own] = priv
        if trace is not None:
            trace.setdefault("block", {})[p] = own

    # Redistribution, then the cyclic phase: processor p owns indices = p mod m.
    # In its private copy, global index m*i + p sits at i, so a column of
    # length L (L/2 >= m) holds L/m private elements, the butterfly partner
    # of private position i is i + L/(2m), and the global row of private row
    # r' is m*r' + p: only those L/(2m) weights are needed.
    for p in range(m):
        own = np.arange(p, n, m)
        priv = y[own].copy()
        for q in range(breakpoint, t + 1):
            L = 1 << q
            rows = m * np.arange(L // (2 * m)) + p
            _stage_on_columns(priv.reshape(n // L, L // m), _weights(rows, L, sign))
        y[own] = priv
        if trace is not None:
            trace.setdefault("cyclic", {})[p] = own
    return y

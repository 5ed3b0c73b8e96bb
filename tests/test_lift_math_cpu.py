"""The index maps and weights of the two- and three-level lifts, written out
in NumPy from their definitions, against the FP64 oracle (CPU only).

These pin the decompositions the GPU passes implement -- which lines each
pass transforms, which weight it applies, and where each result is stored --
independently of the kernels: a dropped weight, a swapped stride or a wrong
output index map fails here before any GPU run.  The per-line transforms are
the oracle's own DFT of each line (the oracle is the reference for the
transform itself; what is under test is the composition).
"""
import numpy as np
import pytest

import datagen
import oracle


def w(e, n, sign):
    return np.exp(sign * 2j * np.pi * (np.asarray(e) % n) / n)


def line_fft(lines, sign):
    return oracle.fft_batch(np.ascontiguousarray(lines), sign)


def two_level(x, log2p, sign):
    """n = p q: q-point column transforms (stride p), weight w_n^(j1 k2),
    p-point row transforms, output X[k2 + q k1]."""
    n = x.size
    p = 1 << log2p
    q = n // p
    A = x.reshape(q, p)                    # A[j2][j1] = x[j1 + p j2]
    Y = line_fft(A.T, sign)                # Y[j1][k2]
    j1 = np.arange(p)[:, None]
    k2 = np.arange(q)[None, :]
    Y = Y * w(j1 * k2, n, sign)
    Z = line_fft(Y.T, sign)                # Z[k2][k1]
    out = np.empty(n, complex)
    k1 = np.arange(p)[None, :]
    out[(k2.T + q * k1).ravel()] = Z.ravel()
    return out


def factors(t):
    """The library's three-level split: log2 n3 = ceil(t/3), log2 n1 =
    ceil((t - log2 n3)/2), n2 the rest."""
    l3 = (t + 2) // 3
    l1 = (t - l3 + 1) // 2
    return l1, t - l3 - l1, l3


def three_level(x, sign, split=None):
    """n = n1 n2 n3, j = j1 + n1 j2 + n1 n2 j3, k = k3 + n3 k2 + n2 n3 k1.
    Pass A: n3-point transforms along j3, times w_n^(n1 j2 k3), stored where
    j3 was; pass B: n2-point transforms along j2, times w_n^(j1 (k3 + n3 k2)),
    stored where j2 was; pass C: n1-point transforms of the contiguous rows,
    stored at k3 + n3 k2 + n2 n3 k1."""
    n = x.size
    l1, l2, l3 = split or factors(int(np.log2(n)))
    n1, n2, n3 = 1 << l1, 1 << l2, 1 << l3
    V = x.reshape(n3, n2, n1).astype(complex)             # V[j3][j2][j1]
    # pass A (lines over (j2, j1), points along j3)
    V = np.moveaxis(line_fft(np.moveaxis(V, 0, -1).reshape(-1, n3), sign).reshape(n2, n1, n3), -1, 0)
    j2 = np.arange(n2)[None, :, None]
    k3 = np.arange(n3)[:, None, None]
    V = V * w(n1 * j2 * k3, n, sign)                      # V[k3][j2][j1]
    # pass B (lines over (k3, j1), points along j2)
    V = np.moveaxis(line_fft(np.moveaxis(V, 1, -1).reshape(-1, n2), sign).reshape(n3, n1, n2), -1, 1)
    j1 = np.arange(n1)[None, None, :]
    k2 = np.arange(n2)[None, :, None]
    V = V * w(j1 * (k3 + n3 * k2), n, sign)               # V[k3][k2][j1]
    # pass C (contiguous rows over (k3, k2), points along j1)
    Z = line_fft(V.reshape(-1, n1), sign).reshape(n3, n2, n1)   # Z[k3][k2][k1]
    out = np.empty(n, complex)
    k1 = np.arange(n1)[None, None, :]
    out[(k3 + n3 * k2 + n2 * n3 * k1).ravel()] = Z.ravel()
    return out


@pytest.mark.parametrize("sign", [-1, 1])
@pytest.mark.parametrize("t,log2p", [(6, 3), (9, 4), (10, 5), (12, 1), (12, 11), (14, 7)])
def test_two_level_composition(t, log2p, sign):
    x = datagen.signals(1 << t, 1, np.complex128, "normal", 70 + t)[0]
    ref = oracle.fft(x, sign)
    assert oracle.rel_l2(two_level(x, log2p, sign), ref) <= 1e-13


@pytest.mark.parametrize("sign", [-1, 1])
@pytest.mark.parametrize("t", [6, 9, 12, 15, 16, 17, 18])
def test_three_level_composition(t, sign):
    x = datagen.signals(1 << t, 1, np.complex128, "normal", 80 + t)[0]
    ref = oracle.fft(x, sign)
    assert oracle.rel_l2(three_level(x, sign), ref) <= 1e-13


@pytest.mark.parametrize("split", [(1, 1, 1), (1, 2, 3), (3, 2, 1), (2, 4, 3), (5, 1, 2)])
def test_three_level_any_split(split):
    t = sum(split)
    x = datagen.signals(1 << t, 1, np.complex128, "uniform", 90 + t)[0]
    assert oracle.rel_l2(three_level(x, -1, split), oracle.fft(x, -1)) <= 1e-13


def test_factor_rule():
    """Near-equal factors with n3 >= n1 >= n2, summing to t; 2^24 = 256^3."""
    for t in range(15, 34):
        l1, l2, l3 = factors(t)
        assert l1 + l2 + l3 == t and l3 >= l1 >= l2 and l3 - l2 <= 1
    assert factors(24) == (8, 8, 8)


def test_dropping_a_weight_is_detected():
    """The composition test is sensitive: without the weights, or with
    weight exponents of the wrong stride (three times too large), the
    result is far from the DFT."""
    t = 12
    x = datagen.signals(1 << t, 1, np.complex128, "normal", 99)[0]
    ref = oracle.fft(x, -1)
    saved = w
    try:
        globals()["w"] = lambda e, n, sign: np.ones(np.shape(e), complex)
        assert oracle.rel_l2(three_level(x, -1), ref) > 0.1
        globals()["w"] = lambda e, n, sign: saved(3 * np.asarray(e), n, sign)
        assert oracle.rel_l2(three_level(x, -1), ref) > 0.1
    finally:
        globals()["w"] = saved

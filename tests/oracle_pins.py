"""Pins for the FP64 oracle: checks that fix it to what the paper and the
mathematics say, rather than to itself.

Each ``pin_*`` function takes an :class:`oracle.Oracle` and raises
``AssertionError`` on a mismatch.  ``tests/test_oracle_pins.py`` runs them on
the oracle; ``tests/test_oracle_mutants.py`` runs them on deliberately broken
builds of the oracle source and requires every broken build to fail at least
one of them.

The definition being pinned is Section 2.1, Fig. 2.1 of the paper:
X[k] = sum_j x[j] w_n^(sign*j*k), w_n = exp(2 pi i/n), n = 2^t, t >= 1,
unnormalized, natural-order output.
"""
from __future__ import annotations

import os

import numpy as np

import datagen
from oracle import rel_l2
from paper_plan import breakpoint_range, partitioned_fft, staged_fft

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "dft_by_hand.txt")


def _cvec(text: str) -> np.ndarray:
    vals = []
    for tok in text.split():
        re, im = tok.split(",")
        vals.append(complex(float(re), float(im)))
    return np.array(vals, dtype=np.complex128)


def golden_cases():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, n, sign, xs, Xs = [s.strip() for s in line.split("|")]
            x, X = _cvec(xs), _cvec(Xs)
            assert x.size == int(n) == X.size, name
            cases.append((name, int(sign), x, X))
    return cases


def _rand(n, seed, dist="normal"):
    return datagen.signals(n, 1, np.complex128, dist, seed)[0]


# --- the definition (O(n^2)) ------------------------------------------------

def pin_dft_golden(o):
    """Hand-worked examples (tests/golden/dft_by_hand.txt)."""
    for name, sign, x, X in golden_cases():
        got = o.dft(x, sign)
        assert np.max(np.abs(got - X)) < 1e-14, (name, got, X)


def pin_dft_delta_and_tone(o):
    """e_j -> w^(sign*j*k); pure tone w^(-sign*a*j) -> n * delta_{k,a}."""
    for n in (2, 8, 32):
        for sign in (-1, 1):
            k = np.arange(n)
            for j in (0, 1, n - 1):
                e = np.zeros(n, complex)
                e[j] = 1
                want = np.exp(sign * 2j * np.pi * ((j * k) % n) / n)
                assert np.max(np.abs(o.dft(e, sign) - want)) < 1e-13, (n, sign, j)
            for a in (0, 1, n // 2 + 1 if n > 2 else 1):
                tone = np.exp(-sign * 2j * np.pi * ((a * k) % n) / n)
                want = np.zeros(n, complex)
                want[a] = n
                assert np.max(np.abs(o.dft(tone, sign) - want)) < 1e-12, (n, sign, a)


def pin_dft_library(o):
    """Special case that reduces to a library routine: numpy.fft (pocketfft)."""
    for n in (2, 4, 16, 64, 128):
        x = _rand(n, 100 + n)
        assert rel_l2(o.dft(x, -1), np.fft.fft(x)) < 1e-13, n
        assert rel_l2(o.dft(x, 1), n * np.fft.ifft(x)) < 1e-13, n


# --- the FFT (Fig. 2.1) -------------------------------------------------------

def pin_fft_golden(o):
    for name, sign, x, X in golden_cases():
        got = o.fft(x, sign)
        assert np.max(np.abs(got - X)) < 1e-14, (name, got, X)


def pin_fft_brute_force(o):
    """Every n = 2..256 (and 512) against the definition, both signs."""
    for t in range(1, 10):
        n = 1 << t
        for sign in (-1, 1):
            x = _rand(n, 7 * n + (sign > 0), "uniform")
            assert rel_l2(o.fft(x, sign), o.dft(x, sign)) < 1e-13, (n, sign)


def pin_fft_library(o):
    for t in (1, 3, 10, 14, 17):
        n = 1 << t
        x = _rand(n, 31 + t)
        assert rel_l2(o.fft(x, -1), np.fft.fft(x)) < 1e-13, n
        assert rel_l2(o.fft(x, 1), n * np.fft.ifft(x)) < 1e-13, n


def pin_fft_closed_forms(o):
    """delta_0 -> all ones exactly; ones -> n delta_0; n = 2 closed form."""
    for t in (1, 4, 11):
        n = 1 << t
        d = np.zeros(n, complex)
        d[0] = 1
        for sign in (-1, 1):
            assert np.array_equal(o.fft(d, sign), np.ones(n, complex)), n
            want = np.zeros(n, complex)
            want[0] = n
            assert np.max(np.abs(o.fft(np.ones(n, complex), sign) - want)) < 1e-9 * n, n
    x = np.array([0.25 - 1.5j, -2.0 + 0.5j])
    for sign in (-1, 1):
        assert np.array_equal(o.fft(x, sign), np.array([x[0] + x[1], x[0] - x[1]]))


def pin_fft_tone(o):
    for t in (3, 8, 12):
        n = 1 << t
        j = np.arange(n)
        for sign in (-1, 1):
            for a in (1, n // 3, n - 1):
                tone = np.exp(-sign * 2j * np.pi * ((a * j) % n) / n)
                want = np.zeros(n, complex)
                want[a] = n
                assert np.max(np.abs(o.fft(tone, sign) - want)) < 1e-10 * n, (n, a)


def pin_fft_properties(o):
    """Parseval, linearity, shift theorem, round trip, Hermitian symmetry."""
    for t in (5, 12, 16):
        n = 1 << t
        x = _rand(n, 1000 + t)
        y = _rand(n, 2000 + t)
        k = np.arange(n)
        for sign in (-1, 1):
            X = o.fft(x, sign)
            # Parseval: sum |X|^2 = n sum |x|^2
            assert abs(np.vdot(X, X).real / (n * np.vdot(x, x).real) - 1) < 1e-13
            # linearity with complex coefficients
            a, b = 0.3 - 1.1j, -2.5 + 0.25j
            lhs = o.fft(a * x + b * y, sign)
            assert rel_l2(lhs, a * X + b * o.fft(y, sign)) < 1e-13
            # shift theorem: roll by s multiplies X_k by w^(sign*s*k)
            for s in (1, 5, n // 2 + 3):
                want = np.exp(sign * 2j * np.pi * ((s * k) % n) / n) * X
                assert rel_l2(o.fft(np.roll(x, s), sign), want) < 1e-12, (n, s)
            # round trip: F_{-s} F_s x = n x
            assert rel_l2(o.fft(X, -sign), n * x) < 1e-13
        # Hermitian symmetry of a real input: X[n-k] = conj X[k]
        r = x.real.astype(complex)
        R = o.fft(r, -1)
        assert np.max(np.abs(R[(-k) % n] - np.conj(R))) < 1e-12 * np.max(np.abs(R))


def pin_fft_batch(o):
    x = datagen.signals(256, 9, np.complex128, "normal", 5)
    got = o.fft_batch(x, -1, threads=3)
    for b in range(x.shape[0]):
        assert rel_l2(got[b], o.dft(x[b], -1)) < 1e-13, b


def pin_paper_plan(o):
    """The paper's iterative stage loop and its block/cyclic plan (Section 4)
    reach the same result as the oracle for every valid breakpoint.  The
    paper's weights carry the +1 exponent, so its transform is sign = +1."""
    for t in (2, 4, 6, 8):
        n = 1 << t
        x = _rand(n, 300 + t)
        ref = o.fft(x, 1)
        assert rel_l2(staged_fft(x, 1), ref) < 1e-13, n
        assert rel_l2(staged_fft(x, -1), o.fft(x, -1)) < 1e-13, n
        m = 1
        while n // m >= m:
            lo, hi = breakpoint_range(n, m)
            for bp in range(lo, hi + 1):
                got = partitioned_fft(x, m, bp, 1)
                assert rel_l2(got, ref) < 1e-13, (n, m, bp)
            m *= 2


def pin_four_step_identity(o):
    """The lift used by the GPU path: n = p*q, j = j1 + p*j2, k = k2 + q*k1,
    Y[j1,k2] = DFT_q over j2 of x[j1 + p*j2], times w_n^(sign*j1*k2), then
    X[k2 + q*k1] = DFT_p over j1 of Y[j1,k2] -- equals the n-point DFT."""
    for p, q in ((32, 32), (16, 32), (32, 16), (4, 64), (2, 8), (64, 4)):
        n = p * q
        x = _rand(n, p * 1000 + q)
        for sign in (-1, 1):
            A = x.reshape(q, p)              # A[j2, j1] = x[j1 + p*j2]
            Y = np.stack([o.fft(A[:, j1], sign) for j1 in range(p)])   # Y[j1, k2]
            j1 = np.arange(p)[:, None]
            k2 = np.arange(q)[None, :]
            Y = Y * np.exp(sign * 2j * np.pi * ((j1 * k2) % n) / n)
            Z = np.stack([o.fft(Y[:, c], sign) for c in range(q)])    # Z[k2, k1]
            X = Z.T.reshape(n)               # X[k2 + q*k1] = Z[k2, k1]
            assert rel_l2(X, o.fft(x, sign)) < 1e-13, (p, q, sign)


ALL_PINS = [
    pin_dft_golden, pin_dft_delta_and_tone, pin_dft_library,
    pin_fft_golden, pin_fft_brute_force, pin_fft_library, pin_fft_closed_forms,
    pin_fft_tone, pin_fft_properties, pin_fft_batch, pin_paper_plan,
    pin_four_step_identity,
]


def failing_pins(o) -> list[str]:
    """Names of the pins that fail (or raise) for oracle ``o``."""
    bad = []
    for pin in ALL_PINS:
        try:
            pin(o)
        except Exception:  # noqa: BLE001 - any failure counts
            bad.append(pin.__name__)
    return bad

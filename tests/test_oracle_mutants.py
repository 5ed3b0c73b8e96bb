"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case copies ``oracle/oracle.c``, makes one plausible mistake in the copy
(a dropped term, a wrong sign, a wrong index, a transposed operand), builds it
with gcc into a temporary directory and runs the full pin battery against the
broken build.  Every mistake must make at least one pin fail.  The oracle
source itself is never modified.
"""
import os
import subprocess

import pytest

import oracle
import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, exact text in oracle.c, replacement).  All stay in bounds.
MUTANTS = [
    ("weight_sign_flipped", "w[2 * e + 1] = (double)sign * sin(a);",
     "w[2 * e + 1] = -(double)sign * sin(a);"),
    ("cmul_dropped_term", "double cr = wr * orr - wi * oi;", "double cr = wr * orr;"),
    ("cmul_transposed_operand", "double ci = wr * oi + wi * orr;",
     "double ci = wr * orr + wi * oi;"),
    ("butterfly_wrong_sign", "out[2 * (r + h)] = er - cr;", "out[2 * (r + h)] = er + cr;"),
    ("butterfly_dropped_term", "out[2 * r + 1] = ei + ci;", "out[2 * r + 1] = ei;"),
    ("weight_wrong_index", "wi = wtab[2 * (r * step) + 1];",
     "wi = wtab[2 * ((r * step) / 2) + 1];"),
    ("split_wrong_subsequence", "fft_level(x, 2 * s, out, h, wtab, n);",
     "fft_level(x + 2 * s, 2 * s, out, h, wtab, n);"),
    ("dft_exponent_off_by_one", "uint64_t e = ((uint64_t)j * (uint64_t)k) % (uint64_t)n;",
     "uint64_t e = ((uint64_t)j * (uint64_t)(k + 1)) % (uint64_t)n;"),
    ("dft_wrong_sign", "re += xr * wr - xi * wi;", "re += xr * wr + xi * wi;"),
    ("dft_transposed_operand", "im += xr * wi + xi * wr;", "im += xr * wr + xi * wi;"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site for %s not unique in oracle.c" % name
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", str(lib),
                    str(mutated), "-lm", "-lpthread"], check=True)
    bad = oracle_pins.failing_pins(oracle.load_library(str(lib)))
    assert bad, "planted mistake %s passed every pin" % name

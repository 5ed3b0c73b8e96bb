"""The FP64 oracle against its pins (CPU only)."""
import pytest

import oracle
import oracle_pins


@pytest.fixture(scope="module")
def o():
    return oracle.default()


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(o, pin):
    pin(o)


def test_golden_file_has_cases():
    assert len(oracle_pins.golden_cases()) >= 8


def test_oracle_rejects_bad_arguments(o):
    import numpy as np
    for n in (0, 1, 3, 6, 12):
        with pytest.raises(ValueError):
            o.fft(np.zeros(n, complex), -1)
    with pytest.raises(ValueError):
        o.fft(np.zeros(8, complex), 2)
    with pytest.raises(ValueError):
        o.dft(np.zeros(8, complex), 0)

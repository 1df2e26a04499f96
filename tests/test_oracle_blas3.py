"""The oracle's level-3 routines (dsyrk, dtrmm, dtrsm) against their pins (CPU only)."""
import pytest

import blas3_pins


@pytest.mark.parametrize("pin", blas3_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_blas3_pin(pin):
    pin(None)

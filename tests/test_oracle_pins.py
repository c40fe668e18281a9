"""The FP64 oracle against what the paper and the mathematics fix.

Every pin is described in ``tests/pins.py``.  These run on the CPU only.
"""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_oracle_pin(pin):
    pin()

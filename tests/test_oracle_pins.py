"""Pin the CPU oracle to the paper and to mathematics (no GPU)."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin, olib):
    pin(olib)

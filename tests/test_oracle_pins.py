"""The oracle against the paper and the mathematics (see oracle_pins.py)."""
import pytest

import oracle_pins as pins


@pytest.mark.parametrize("pin", pins.ALL, ids=[f.__name__ for f in pins.ALL])
def test_pin(oracle_mod, pin):
    pin(oracle_mod)

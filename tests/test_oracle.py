"""The CPU oracle against its pins (no GPU)."""
import pytest

import filter_pins
import map_pins
import nbd_pins
import oracle_pins as pins


@pytest.mark.parametrize("pin", pins.ALL_PINS + nbd_pins.ALL_NBD_PINS + filter_pins.ALL_FILTER_PINS + map_pins.ALL_MAP_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin, oracle_lib):
    pin(oracle_lib)

"""The morphology oracle against its pins (tests/pins_morph.py)."""
import pytest

import pins_morph


@pytest.mark.parametrize("pin", pins_morph.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin()

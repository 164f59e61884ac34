"""The two-dimensional oracle against its pins (tests/pins2d.py)."""
import pytest

import pins2d


@pytest.mark.parametrize("pin", pins2d.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin()

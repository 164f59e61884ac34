"""The CPU oracle against its pins (closed forms, limits, library routines,
invariants and an independent dynamic programme)."""
import pytest

import oracle
import pins

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.mark.parametrize("pin", [p for p in pins.ALL_PINS if p not in pins.MODE_PINS], ids=lambda p: p.__name__)
def test_pin(pin):
    pin()


@pytest.mark.parametrize("mode", [oracle.MODE_DIRECT, oracle.MODE_PREFIX], ids=["direct", "prefix"])
@pytest.mark.parametrize("pin", pins.MODE_PINS, ids=lambda p: p.__name__)
def test_mode_pin(pin, mode):
    pin(mode=mode)

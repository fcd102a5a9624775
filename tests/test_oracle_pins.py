"""The CPU oracle against its pins (closed forms, library routines, brute
force, exact-arithmetic equivalences); see tests/pins.py."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()

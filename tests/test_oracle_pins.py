"""The CPU oracle against closed forms, invariants, brute force and the
hand-worked golden cases (CPU only)."""
import pytest

from oracle import evis_oracle as o
import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(o)

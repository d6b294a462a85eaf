"""The FP64 oracle against its pins (brute force, library special cases,
closed-form invariants of the local linear model).  CPU only."""
import pytest

import pins
from oracle import oracle


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin(oracle.default())

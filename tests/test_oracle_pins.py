"""The FP64 oracle against closed forms, invariants and brute force (CPU)."""

import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()

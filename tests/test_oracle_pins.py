"""The oracle against its pins (hand-derived closed forms, special cases, a
library matrix product, an independent brute-force simulator, invariants)."""
import pytest

from tests import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()

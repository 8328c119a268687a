"""The FP64 oracle against facts fixed by the paper and by mathematics (CPU only)."""
import pytest

from tests.oracle_pins import PINS


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_pin(orc, pin):
    pin(orc, orc.load())

"""The oracle against facts fixed outside of it (see tests/pins.py)."""

import pytest

from oracle import dbscan_brute, dbscan_o1
from tests.pins import ALL_PINS

IMPLS = {"O0_brute": dbscan_brute, "O1_c": dbscan_o1}


@pytest.mark.parametrize("impl", sorted(IMPLS))
@pytest.mark.parametrize("pin", sorted(ALL_PINS))
def test_oracle_pin(pin, impl):
    fails = ALL_PINS[pin](IMPLS[impl])
    assert not fails, "\n".join(fails)

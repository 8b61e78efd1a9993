"""The oracle against facts fixed by the paper and by mathematics (CPU only)."""
import pytest

import oracle
from tests import oracle_pins as pins


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(ora, check):
    check(ora)

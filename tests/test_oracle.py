"""The CPU oracle against its pins (closed forms, dense products, parameter shift, ...)."""
import os

import pytest

import oracle_pins
from oracle.oracle import LIB_PATH, Oracle, build


@pytest.fixture(scope="module")
def orc():
    if not os.path.exists(LIB_PATH):
        build()
    return Oracle()


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)

"""The CPU oracle against hand-derived cases, closed forms and statistics."""
import pytest

import pins


@pytest.mark.parametrize("check", pins.ALL, ids=lambda f: f.__name__)
def test_pin(orc, check):
    check(orc.load())


def test_run_invariants(orc):
    pins.check_run_invariants(orc.load())


def test_step_rate_equation(orc):
    pins.check_step_rate_equation(orc.load())


def test_chain_consumption(orc):
    pins.check_chain_consumption(orc.load())

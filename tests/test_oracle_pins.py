"""CPU pins of the FP64 oracle (no GPU): each check compares the oracle with
a fact fixed by the paper or by the mathematics (see oracle_pins.py)."""
import pytest

import oracle_pins as P
from oracle import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def lib():
    return O.load()


@pytest.mark.parametrize("check", P.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(lib, check):
    check(lib)


@pytest.mark.parametrize("check", [P.check_lattice, P.check_feq_moments,
                                   P.check_geq_moments, P.check_source_moments,
                                   P.check_recover], ids=lambda c: c.__name__)
def test_pin_d3q19(lib, check):
    check(lib, W.D3Q19)


def test_flat_interface(lib):
    P.check_flat_interface(lib)


def test_laplace_law(lib):
    P.check_laplace(lib)

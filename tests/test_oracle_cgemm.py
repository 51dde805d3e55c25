"""Pins of the complex dd oracle (Cgemm): the manual's worked Cgemm example in
both of its printed forms, exact rational arithmetic on small random cases in
all nine op combinations, bit-exact identities (transposed and conjugated
copies, real data reducing to the real oracle, quick returns, beta = 0, the
identity matrix) and the BLAS argument positions."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


def test_cgemm_worked_example(lib):
    pins.check_cgemm_worked_example(lib)


@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_cgemm_exact_rational(lib, dist):
    pins.check_exact_cgemm(lib, dist=dist)


def test_cgemm_identities(lib):
    pins.check_cgemm_identities(lib)


def test_cgemm_info_codes(lib):
    pins.check_cgemm_info_codes(lib)

"""Pins of the dd division, square root and Cholesky (Rpotrf) oracle: exact
rationals within the published error bounds, exact special cases, integer
factorisations reproduced exactly, the entrywise backward-error bound against
exact arithmetic, uplo U as the bitwise transpose of uplo L, and LAPACK's
info codes (argument errors and the order of the first non-positive pivot)."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


def test_div_sqrt(lib):
    pins.check_div_sqrt(lib)


def test_potrf_exact_integer(lib):
    pins.check_potrf_exact_integer(lib)


def test_potrf_residual(lib):
    pins.check_potrf_residual(lib)


def test_potrf_transpose_and_info(lib):
    pins.check_potrf_transpose_and_info(lib)

"""Pins of the quad-double Rgemm oracle: its exact accumulator rounds to the
greedy nearest qd exactly as rational arithmetic does, every entry of small
products equals the exactly rounded result in all op forms, the manual's
worked Rgemm example comes out exact, BLAS semantics and argument positions
hold, and the tolerance unit is the manual's qd epsilon."""
from fractions import Fraction

import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


def test_qd_epsilon_reading():
    """Table "rlamch_qd" prints eps to 64 digits; they agree with 2^-209 to
    about 14 significant digits (the printout is binary64-accurate beyond
    that, as for dd), so the tolerance unit is 2^-209, precision 2^-208,
    212 mantissa bits."""
    vals = {}
    with open(pins.os.path.join(pins.GOLDEN, "rlamch_qd.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = Fraction(v)
    assert abs(vals["E"] / Fraction(1, 2 ** 209) - 1) < Fraction(1, 2 ** 45)
    assert abs(vals["P"] / Fraction(1, 2 ** 208) - 1) < Fraction(1, 2 ** 45)
    assert vals["N"] == 212


def test_qd_round(lib):
    pins.check_qd_round(lib)


@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_qgemm_exact(lib, dist):
    pins.check_qgemm_exact(lib, dist=dist)


def test_qgemm_semantics(lib):
    pins.check_qgemm_semantics(lib)

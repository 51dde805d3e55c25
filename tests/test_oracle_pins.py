"""The CPU oracle against its pins (no GPU): worked example, exact rational
arithmetic, BLAS error codes, bit-exact identities, split-form exactness."""
import ctypes
import ctypes.util

import numpy as np
import pytest

import oracle
import pins
import workloads as W
from oracle.compare import bits


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


def test_worked_example(lib):
    pins.check_worked_example(lib)


def test_primitives_exact(lib):
    pins.check_primitives(lib)


@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_gemm_vs_exact(lib, dist):
    pins.check_exact_gemm(lib, dist=dist)


def test_gemm_vs_exact_medium(lib):
    # one larger case with wide exponents: k = 24 spans several "tiles" of terms
    pins.check_exact_gemm(lib, seeds=[9], dist="wide", sizes=[(5, 4, 24)])


@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_syrk_vs_exact(lib, dist):
    pins.check_exact_syrk(lib, dist=dist)


def test_info_codes(lib):
    pins.check_info_codes(lib)


def test_identities(lib):
    pins.check_identities(lib)


def test_ozaki_split_exact(lib):
    pins.check_ozaki_split_exact(lib)
    pins.check_ozaki_split_exact(lib, dist="uniform", nslices=10)


def test_ozaki_gemm_exact(lib):
    pins.check_ozaki_gemm_exact(lib)


def test_tolerance_unit_is_rlamch_eps():
    """The tolerance unit 2^-104 is the manual's Rlamch('E') for dd.

    The table prints 32 digits, of which the first 16 agree with 2^-104 and
    the rest differ at the 1e-16 relative level (the printout is only good
    to binary64 accuracy there); so the reading is eps = 2^-104 exactly,
    precision = 2 eps, 106 mantissa bits."""
    from fractions import Fraction
    vals = {}
    with open(pins.os.path.join(pins.GOLDEN, "rlamch_dd.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = Fraction(v)
    from oracle.compare import EPS_DD
    assert abs(vals["E"] / Fraction(EPS_DD) - 1) < Fraction(1, 2 ** 50)
    assert abs(vals["P"] / Fraction(2 * EPS_DD) - 1) < Fraction(1, 2 ** 50)
    assert vals["N"] == 106


def test_thread_count_independent(lib):
    gomp = ctypes.CDLL(ctypes.util.find_library("gomp") or "libgomp.so.1")
    c = W.gemm_case(7000, "T", "N", 37, 29, 41)
    outs = []
    for nt in (1, 3, 8):
        gomp.omp_set_num_threads(nt)
        C = (c["C"][0].copy(), c["C"][1].copy())
        assert oracle.rgemm("T", "N", 37, 29, 41, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"],
                            c["beta"], C, c["ldc"], lib=lib) == 0
        outs.append(C)
    gomp.omp_set_num_threads(8)
    for C in outs[1:]:
        assert np.array_equal(bits(C[0]), bits(outs[0][0]))
        assert np.array_equal(bits(C[1]), bits(outs[0][1]))


def test_entries_match_full(lib):
    """The sampled-entry routines return exactly the full routines' values."""
    c = W.gemm_case(7100, "N", "T", 33, 21, 17)
    C = (c["C"][0].copy(), c["C"][1].copy())
    oracle.rgemm("N", "T", 33, 21, 17, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"], c["beta"],
                 C, c["ldc"], lib=lib)
    rng = np.random.default_rng(1)
    ii, jj = rng.integers(0, 33, 50), rng.integers(0, 21, 50)
    h, l = oracle.rgemm_entries("N", "T", 33, 21, 17, c["alpha"], c["A"], c["lda"], c["B"],
                                c["ldb"], c["beta"], c["C"], c["ldc"], ii, jj, lib=lib)
    idx = ii + jj * c["ldc"]
    assert np.array_equal(h, C[0][idx]) and np.array_equal(l, C[1][idx])
    s = W.syrk_case(7101, "L", "T", 30, 12)
    C = (s["C"][0].copy(), s["C"][1].copy())
    oracle.rsyrk("L", "T", 30, 12, s["alpha"], s["A"], s["lda"], s["beta"], C, s["ldc"], lib=lib)
    jj = rng.integers(0, 30, 40)
    ii = np.array([rng.integers(j, 30) for j in jj])
    h, l = oracle.rsyrk_entries("L", "T", 30, 12, s["alpha"], s["A"], s["lda"], s["beta"],
                                s["C"], s["ldc"], ii, jj, lib=lib)
    idx = ii + jj * s["ldc"]
    assert np.array_equal(h, C[0][idx]) and np.array_equal(l, C[1][idx])


def test_ozaki_converges_to_plain(lib):
    """With enough slices the split form agrees with the plain oracle to the
    dd tolerance, on both input sets; with too few it does not."""
    from oracle.compare import ratio
    for dist, s_ok in (("uniform", 16), ("wide", 22)):
        c = W.gemm_case(7200, "N", "N", 40, 36, 64, dist=dist)
        P = (c["C"][0].copy(), c["C"][1].copy())
        oracle.rgemm("N", "N", 40, 36, 64, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"],
                     c["beta"], P, c["ldc"], lib=lib)
        idx = (np.arange(40)[:, None] + np.arange(36)[None, :] * c["ldc"]).ravel()
        for s, ok in ((s_ok, True), (6, False)):
            Z = (c["C"][0].copy(), c["C"][1].copy())
            oracle.ozaki_rgemm("N", "N", 40, 36, 64, c["alpha"], c["A"], c["lda"], c["B"],
                               c["ldb"], c["beta"], Z, c["ldc"], s,
                               *oracle.int8_digit_widths(64, s), oracle.INT8_QMAX, lib=lib)
            r = ratio(Z[0][idx], Z[1][idx], P[0][idx], P[1][idx], 64)
            assert (r <= 8.0) == ok, (dist, s, r)

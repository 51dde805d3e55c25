"""Pins of the modular split-form oracle (oracle/crt.py) against what the
mathematics fixes: a hand-derived moduli list, pairwise coprimality and the
greedy rule, the bound that fixes P, the rounding of each dd entry to its
integer (checked with exact rationals), congruence and range of the
residues, Chinese remaindering of random integers, the residue route against
the plain big-integer matrix product, and the final result against the exact
product of the dd inputs within the rounding bound of the integer grids.
A second set plants plausible mistakes in copies of the oracle and checks
that these pins catch each one.  CPU only."""
import importlib.util
import os
import random
import tempfile
from fractions import Fraction
from math import gcd

import numpy as np
import pytest

from oracle import crt as CRT

# Moduli by hand: from 256 down, skipping 254, 252, 250, 248, 246, 244, 242,
# 240, ... (even), 249 = 3*83 and 243 (3 | 255), 245 = 5*7^2 and 235 = 5*47
# (5 | 255), 231 = 3*7*11 (3), 221 = 13*17 (17 | 255), 225, 219 = 3*73 ...;
# 217 = 7*31 is coprime to everything before it.
HAND_MODULI = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217]


def _dd_matrix(rng, rows, cols, wide=False):
    """Column-major dd planes (ld = rows) with hi uniform in (-1, 1) or, for
    wide, scaled by 2^e with e in [-20, 20] per entry; lo below ulp(hi)/2."""
    hi = rng.uniform(-1.0, 1.0, rows * cols)
    if wide:
        hi = np.ldexp(hi, rng.integers(-20, 21, rows * cols))
    lo = hi * rng.uniform(-1.0, 1.0, rows * cols) * 2.0 ** -54
    hi, lo = hi + lo, lo - ((hi + lo) - hi)       # renormalise the pair
    return hi, lo


def check_moduli(crt):
    assert crt.moduli(len(HAND_MODULI)) == HAND_MODULI
    ms = crt.moduli(crt.MAX_MODULI)
    for i, a in enumerate(ms):
        for b in ms[:i]:
            assert gcd(a, b) == 1
    # greedy: every skipped integer shares a factor with an earlier modulus
    for x in range(ms[-1] + 1, 257):
        if x not in ms:
            assert any(gcd(x, q) > 1 for q in ms if q > x)
    assert all(2 <= m <= 256 for m in ms)


def check_exponent(crt):
    for count in range(1, crt.MAX_MODULI + 1):
        M = 1
        for m in crt.moduli(count):
            M *= m
        for k in (1, 2, 3, 100, 1024, 1025, 8192, 131071):
            p = crt.exponent(k, count)
            k2 = 1 << max(0, (k - 1).bit_length())
            if p is None:
                assert 4 * k2 * 4 > M      # no P >= 1 fits
                continue
            assert 1 <= p <= crt.MAX_BITS
            assert 4 * k * 2 ** (2 * p) <= M
            if p < crt.MAX_BITS:
                # the largest such P for the power of two at or above k
                assert 4 * k2 * 2 ** (2 * p + 2) > M


def check_integers(crt, rng):
    for wide in (False, True):
        hi, lo = _dd_matrix(rng, 7, 33, wide)
        hi, lo = hi.reshape(7, 33), lo.reshape(7, 33)
        hi[3] = 0.0
        lo[3] = 0.0
        e = crt.scale_exponents(hi)
        for r in range(7):
            mx = max(abs(float(v)) for v in hi[r])
            if mx == 0:
                assert e[r] == 0
            else:
                assert 2.0 ** (int(e[r]) - 1) <= mx < 2.0 ** int(e[r])
        for p in (20, 61, 95, 104):
            X = crt.integers(hi, lo, e, p)
            for r in range(7):
                for l in range(33):
                    z = (Fraction(float(hi[r, l])) + Fraction(float(lo[r, l]))) \
                        * Fraction(2) ** (p - int(e[r]))
                    assert abs(X[r, l] - z) <= Fraction(1, 2) + Fraction(1, 2 ** 50)
                    assert abs(X[r, l]) <= 2 ** p


def check_residues(crt, rng):
    count = 12
    ints = np.empty((3, 40), dtype=object)
    for idx in np.ndindex(ints.shape):
        ints[idx] = random.Random(int(rng.integers(1 << 30))).randrange(-2 ** 100, 2 ** 100)
    ints[0, 0] = 0
    ints[0, 1] = 128
    ints[0, 2] = -128
    ints[0, 3] = 2 ** 100
    R = crt.residues(ints, count)
    for t, m in enumerate(crt.moduli(count)):
        for idx in np.ndindex(ints.shape):
            r = int(R[(t,) + idx])
            assert (r - ints[idx]) % m == 0
            assert -128 <= r <= 127
            assert abs(r) <= m // 2
    assert int(R[0, 0, 1]) == -128 and int(R[0, 0, 2]) == -128    # modulo 256


def check_reconstruct(crt):
    rnd = random.Random(7)
    for count in (2, 5, 12, 27, 32):
        ms = crt.moduli(count)
        M = 1
        for m in ms:
            M *= m
        for _ in range(40):
            x = rnd.randrange(-(M // 4), M // 4)
            # any representatives: the plain remainders plus random multiples
            prods = [x % m + m * rnd.randrange(-1000, 1000) for m in ms]
            assert crt.reconstruct(prods, count) == x
        assert crt.reconstruct([0] * count, count) == 0
        # arrays: elementwise, the same values
        xs = [rnd.randrange(-(M // 4), M // 4) for _ in range(6)]
        arr = [np.array([x % m for x in xs], dtype=np.int64) for m in ms]
        assert list(crt.reconstruct(arr, count)) == xs


def check_integer_product(crt, rng):
    m, n, k, count = 5, 4, 9, 14
    A = _dd_matrix(rng, m, k)
    B = _dd_matrix(rng, n, k, wide=True)          # op(B) = B^T (transb 'T')
    ea, eb, p, X = crt.integer_product("N", "T", m, n, k, A, m, B, n, count)
    assert p == crt.exponent(k, count)
    ah, al = crt.row_operand("N", m, k, A, m)
    bh, bl = crt.row_operand("N", n, k, B, n)
    Ai = crt.integers(ah, al, ea, p)
    Bi = crt.integers(bh, bl, eb, p)
    plain = Ai.dot(Bi.T)                          # big-integer product
    for i in range(m):
        for j in range(n):
            assert X[i, j] == plain[i, j]


def check_rgemm(crt, rng):
    for (ta, tb, m, n, k, count, wide) in (("N", "N", 6, 5, 11, 27, False),
                                          ("T", "N", 4, 7, 16, 20, True),
                                          ("N", "T", 3, 3, 1, 3, False)):
        A = _dd_matrix(rng, m * k, 1, wide)
        B = _dd_matrix(rng, k * n, 1)
        C = _dd_matrix(rng, m * n, 1)
        lda = m if ta == "N" else k
        ldb = k if tb == "N" else n
        alpha = (0.75, 2.0 ** -60)
        beta = (-1.25, 0.0)
        c0 = (C[0].copy(), C[1].copy())
        out = crt.crt_rgemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta,
                            (C[0].copy(), C[1].copy()), m, count)
        p = crt.exponent(k, count)
        ah, al = crt.row_operand(ta, m, k, A, lda)
        bh, bl = crt.row_operand("T" if tb == "N" else "N", n, k, B, ldb)
        ea, eb = crt.scale_exponents(ah), crt.scale_exponents(bh)
        a = Fraction(alpha[0]) + Fraction(alpha[1])
        b = Fraction(beta[0]) + Fraction(beta[1])
        half = Fraction(1, 2) + Fraction(1, 2 ** 50)
        for i in range(m):
            for j in range(n):
                exact = sum((Fraction(float(ah[i, l])) + Fraction(float(al[i, l])))
                            * (Fraction(float(bh[j, l])) + Fraction(float(bl[j, l])))
                            for l in range(k))
                da = half * Fraction(2) ** (int(ea[i]) - p)
                db = half * Fraction(2) ** (int(eb[j]) - p)
                bound = sum(da * abs(Fraction(float(bh[j, l])) + Fraction(float(bl[j, l])))
                            + db * abs(Fraction(float(ah[i, l])) + Fraction(float(al[i, l])))
                            + da * db for l in range(k))
                cij = Fraction(float(c0[0][i + j * m])) + Fraction(float(c0[1][i + j * m]))
                want = a * exact + b * cij
                got = Fraction(float(out[0][i + j * m])) + Fraction(float(out[1][i + j * m]))
                tol = abs(a) * bound + abs(want) * Fraction(1, 2 ** 104)
                assert abs(got - want) <= tol, (ta, tb, i, j)


def _cdd_matrix(rng, size, wide=False):
    return _dd_matrix(rng, size, 1, wide) + _dd_matrix(rng, size, 1, wide)


def _celem(X, ld, r, c, conj):
    q = r + c * ld
    re = Fraction(float(X[0][q])) + Fraction(float(X[1][q]))
    im = Fraction(float(X[2][q])) + Fraction(float(X[3][q]))
    return re, (-im if conj else im)


def _op_elem(X, ld, trans, i, l, row):
    """op(X)(i, l) for op(A) (row=True) or op(X)(l, i) for op(B)."""
    t = trans.upper()
    if t == "N":
        return _celem(X, ld, i, l, False) if row else _celem(X, ld, l, i, False)
    return _celem(X, ld, l, i, t == "C") if row else _celem(X, ld, i, l, t == "C")


def check_complex_exponents(crt):
    # a row whose imaginary part is zero takes the real part's exponent, and
    # the other way round; an all-zero row gets 0
    rh = np.array([[2.0 ** -30, -2.0 ** -31], [0.0, 0.0], [0.0, 0.0]])
    ih = np.array([[0.0, 0.0], [0.0, 3.0], [0.0, 0.0]])
    assert list(crt.complex_scale_exponents(rh, ih)) == [-29, 2, 0]
    for count in (20, 27, 32):
        for k in (7, 4096, 8192):
            p = crt.exponent(k, count, margin_bits=3)
            if p is not None and p < crt.MAX_BITS:
                M = crt.modulus_product(count)
                k2 = 1 << max(0, (k - 1).bit_length())
                assert 8 * k * 2 ** (2 * p) <= M < 8 * k2 * 2 ** (2 * p + 2)


def check_complex_integer_product(crt, rng):
    m, n, k, count = 4, 3, 6, 20
    for ta, tb in (("N", "N"), ("C", "T"), ("T", "C")):
        A = _cdd_matrix(rng, m * k, wide=True)
        B = _cdd_matrix(rng, k * n)
        lda = m if ta == "N" else k
        ldb = k if tb == "N" else n
        ea, eb, p, XR, XI = crt.complex_integer_product(ta, tb, m, n, k, A, lda, B, ldb, count)
        assert p == crt.exponent(k, count, margin_bits=3)
        # the grid integers of each part, taken element by element
        for i in range(m):
            for j in range(n):
                wr = wi = 0
                for l in range(k):
                    a = _op_elem(A, lda, ta, i, l, True)
                    b = _op_elem(B, ldb, tb, j, l, False)
                    ga = [crt.integers(np.array([[float(v)]]), np.array([[float(v - Fraction(float(v)))]]),
                                       np.array([int(ea[i])]), p)[0, 0] for v in a]
                    gb = [crt.integers(np.array([[float(v)]]), np.array([[float(v - Fraction(float(v)))]]),
                                       np.array([int(eb[j])]), p)[0, 0] for v in b]
                    wr += ga[0] * gb[0] - ga[1] * gb[1]      # the textbook product
                    wi += ga[0] * gb[1] + ga[1] * gb[0]
                assert XR[i, j] == wr and XI[i, j] == wi, (ta, tb, i, j)


def check_cgemm(crt, rng):
    for (ta, tb, m, n, k, count) in (("N", "N", 4, 3, 9, 27), ("C", "T", 3, 4, 5, 22),
                                      ("T", "C", 2, 2, 6, 30), ("C", "C", 3, 2, 4, 25)):
        A = _cdd_matrix(rng, m * k, wide=True)
        B = _cdd_matrix(rng, k * n)
        C = _cdd_matrix(rng, m * n)
        lda = m if ta == "N" else k
        ldb = k if tb == "N" else n
        alpha = ((0.75, 2.0 ** -60), (-0.5, 0.0))
        beta = ((-1.25, 0.0), (0.25, 0.0))
        out = crt.crt_cgemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta,
                            tuple(x.copy() for x in C), m, count)
        p = crt.exponent(k, count, margin_bits=3)
        # exponents by hand: the largest |hi| over both parts of each row
        def exps(rows, get):
            out_e = []
            for r in range(rows):
                mx = max(max(abs(float(v)) for v in get(r, l)) for l in range(k))
                out_e.append(0 if mx == 0 else int(np.frexp(mx)[1]))
            return out_e
        ea = exps(m, lambda r, l: _op_elem(A, lda, ta, r, l, True))
        eb = exps(n, lambda r, l: _op_elem(B, ldb, tb, r, l, False))
        fr = lambda x: Fraction(x[0]) + Fraction(x[1])
        a_r, a_i, b_r, b_i = fr(alpha[0]), fr(alpha[1]), fr(beta[0]), fr(beta[1])
        half = Fraction(1, 2) + Fraction(1, 2 ** 50)
        for i in range(m):
            for j in range(n):
                sr = si = Fraction(0)
                bound = Fraction(0)
                da = half * Fraction(2) ** (ea[i] - p)
                db = half * Fraction(2) ** (eb[j] - p)
                for l in range(k):
                    a = _op_elem(A, lda, ta, i, l, True)
                    b = _op_elem(B, ldb, tb, j, l, False)
                    sr += a[0] * b[0] - a[1] * b[1]
                    si += a[0] * b[1] + a[1] * b[0]
                    bound += 2 * (da * (abs(b[0]) + abs(b[1])) + db * (abs(a[0]) + abs(a[1]))
                                  + 2 * da * db)
                q = i + j * m
                cr = Fraction(float(C[0][q])) + Fraction(float(C[1][q]))
                ci = Fraction(float(C[2][q])) + Fraction(float(C[3][q]))
                want_r = a_r * sr - a_i * si + b_r * cr - b_i * ci
                want_i = a_r * si + a_i * sr + b_r * ci + b_i * cr
                got_r = Fraction(float(out[0][q])) + Fraction(float(out[1][q]))
                got_i = Fraction(float(out[2][q])) + Fraction(float(out[3][q]))
                tol = (abs(a_r) + abs(a_i)) * bound
                assert abs(got_r - want_r) <= tol + abs(want_r) * Fraction(1, 2 ** 104), \
                    (ta, tb, i, j)
                assert abs(got_i - want_i) <= tol + abs(want_i) * Fraction(1, 2 ** 104), \
                    (ta, tb, i, j)


def _qd_matrix(rng, size, wide=False):
    x0 = rng.uniform(-1.0, 1.0, size)
    if wide:
        x0 = np.ldexp(x0, rng.integers(-20, 21, size))
    parts = [x0]
    for _ in range(3):
        parts.append(parts[-1] * rng.uniform(-1.0, 1.0, size) * 2.0 ** -53)
    return parts


def _qd_value(X, q):
    return sum(Fraction(float(p[q])) for p in X)


def check_qd_split(crt, rng):
    for wide in (False, True):
        X = _qd_matrix(rng, 6 * 11, wide)
        parts = [p.reshape(6, 11) for p in X]
        parts[0][2] = 0.0
        for p in parts[1:]:
            p[2] = 0.0
        e = crt.qd_scale_exponents(parts[0])
        ch = crt.qd_chunks(parts, e)
        x1, x0 = crt.qd_split(ch)
        for r in range(6):
            for l in range(11):
                z = sum(Fraction(float(p[r, l])) for p in parts) \
                    * Fraction(2) ** (crt.QD_GRID_BITS - int(e[r]))
                xi = sum(int(np.rint(np.ldexp(float(p[r, l]), crt.QD_GRID_BITS - int(e[r]))))
                         for p in parts)
                assert sum(int(ch[j, r, l]) << (26 * j) for j in range(8)) == xi
                assert x1[r, l] * 2 ** 104 + x0[r, l] == xi
                assert abs(xi - z) <= 2
                assert abs(x1[r, l]) < Fraction(2) ** 105 * Fraction(1001, 1000)
                assert abs(x0[r, l]) < Fraction(2) ** 105 * Fraction(1001, 1000)


def check_qd_count(crt):
    for k in (1, 100, 2048, 8192, 131071):
        k2 = 1 << max(0, (k - 1).bit_length())
        for count in range(20, crt.MAX_MODULI + 1):
            M = crt.modulus_product(count)
            ok = crt.qd_count_ok(k, count)
            # the three sub-products lie in [-M/4, M/4]: 4 k (2 * 2^105.01)^2 <= M
            big = 4 * k2 * (2 ** 106 + 2 ** 99) ** 2
            assert ok == (M.bit_length() - 1 >= 215 + (k2.bit_length() - 1))
            if ok:
                assert big <= M


def check_qd_integer_product(crt, rng):
    m, n, k, count = 3, 4, 7, 31
    A = _qd_matrix(rng, m * k, wide=True)
    B = _qd_matrix(rng, n * k)
    ea, eb, X = crt.qd_integer_product("N", "T", m, n, k, A, m, B, n, count)
    pa = crt.qd_row_operand("N", m, k, A, m)
    pb = crt.qd_row_operand("N", n, k, B, n)
    a1, a0 = crt.qd_split(crt.qd_chunks(pa, ea))
    b1, b0 = crt.qd_split(crt.qd_chunks(pb, eb))
    plain = (a1 * 2 ** 104 + a0).dot((b1 * 2 ** 104 + b0).T)     # big-integer product
    for i in range(m):
        for j in range(n):
            assert X[i, j] == plain[i, j]


def check_qgemm(crt, rng):
    for (ta, tb, m, n, k, count) in (("N", "N", 3, 4, 6, 30), ("T", "T", 2, 3, 5, 31)):
        A = _qd_matrix(rng, m * k, wide=True)
        B = _qd_matrix(rng, k * n)
        C = _qd_matrix(rng, m * n)
        lda = m if ta == "N" else k
        ldb = k if tb == "N" else n
        alpha = (0.75, 2.0 ** -60, 0.0, 0.0)
        beta = (-1.25, 0.0, 0.0, 0.0)
        out = crt.crt_qgemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, [p.copy() for p in C],
                            m, count)
        a = sum(Fraction(x) for x in alpha)
        b = sum(Fraction(x) for x in beta)
        def opa(i, l):
            return _qd_value(A, i + l * lda if ta == "N" else l + i * lda)
        def opb(l, j):
            return _qd_value(B, l + j * ldb if tb == "N" else j + l * ldb)
        ea = [int(np.frexp(max(abs(float(A[0][i + l * lda if ta == "N" else l + i * lda]))
                                  for l in range(k)))[1]) for i in range(m)]
        eb = [int(np.frexp(max(abs(float(B[0][l + j * ldb if tb == "N" else j + l * ldb]))
                                  for l in range(k)))[1]) for j in range(n)]
        for i in range(m):
            for j in range(n):
                da = 2 * Fraction(2) ** (ea[i] - crt.QD_GRID_BITS)
                db = 2 * Fraction(2) ** (eb[j] - crt.QD_GRID_BITS)
                exact = sum(opa(i, l) * opb(l, j) for l in range(k))
                bound = sum(da * abs(opb(l, j)) + db * abs(opa(i, l)) + da * db for l in range(k))
                want = a * exact + b * _qd_value(C, i + j * m)
                got = _qd_value(out, i + j * m)
                assert abs(got - want) <= abs(a) * bound + abs(want) * Fraction(1, 2 ** 210), \
                    (ta, tb, i, j)


def test_moduli():
    check_moduli(CRT)


def test_qd_split_chunks_and_bounds():
    check_qd_split(CRT, np.random.default_rng(18))


def test_qd_moduli_count():
    check_qd_count(CRT)


def test_qd_integer_product_equals_big_integer_product():
    check_qd_integer_product(CRT, np.random.default_rng(19))


def test_qgemm_within_grid_rounding_of_exact_product():
    check_qgemm(CRT, np.random.default_rng(20))


def test_complex_exponents_and_margin():
    check_complex_exponents(CRT)


def test_complex_integer_product_equals_textbook_product():
    check_complex_integer_product(CRT, np.random.default_rng(16))


def test_cgemm_within_grid_rounding_of_exact_product():
    check_cgemm(CRT, np.random.default_rng(17))


def test_exponent():
    check_exponent(CRT)


def test_integers_round_to_nearest():
    check_integers(CRT, np.random.default_rng(11))


def test_residues():
    check_residues(CRT, np.random.default_rng(12))


def test_reconstruct():
    check_reconstruct(CRT)


def test_integer_product_equals_big_integer_product():
    check_integer_product(CRT, np.random.default_rng(13))


def test_rgemm_within_grid_rounding_of_exact_product():
    check_rgemm(CRT, np.random.default_rng(14))


def test_quick_cases():
    rng = np.random.default_rng(15)
    C = _dd_matrix(rng, 6, 1)
    A = _dd_matrix(rng, 6, 1)
    # alpha = 0: C = beta C; k = 0 likewise
    for (alpha, k) in (((0.0, 0.0), 3), ((1.0, 0.0), 0)):
        out = CRT.crt_rgemm("N", "N", 2, 3, k, alpha, A, 2, A, max(k, 1), (2.0, 0.0),
                            (C[0].copy(), C[1].copy()), 2, 20)
        assert np.array_equal(out[0], 2.0 * C[0]) and np.array_equal(out[1], 2.0 * C[1])
    # beta = 0 never reads C
    nan = (np.full(6, np.nan), np.full(6, np.nan))
    out = CRT.crt_rgemm("N", "N", 2, 3, 1, (1.0, 0.0), A, 2, A, 1, (0.0, 0.0), nan, 2, 20)
    assert np.all(np.isfinite(out[0]))
    assert CRT.exponent(8192, 2) is None


# ---- planted mistakes ------------------------------------------------------------------

MUTANTS = [
    ("if all(gcd(m, q) == 1 for q in out):", "if all(gcd(m, q) == 1 for q in out[1:]):",
     "moduli not pairwise coprime"),
    ("p = ((M.bit_length() - 1) - margin_bits - lk) // 2",
     "p = ((M.bit_length() - 1) - lk) // 2", "no margin in P"),
    ("t2 = np.rint((zh - t1) + zl)", "t2 = np.rint(zh - t1)", "low part dropped"),
    ("sh = (p - exps).astype(np.int64)[:, None]", "sh = (p + exps).astype(np.int64)[:, None]",
     "scale sign"),
    ("top = (m - 1) // 2 if m % 2 else m // 2 - 1", "top = (m - 1) // 2 if m % 2 else m // 2",
     "residue 128 out of int8"),
    ("x = x + r * (Mt * pow(Mt, -1, m))", "x = x + r * Mt",
     "weights without the inverse"),
    ("half = (M + 1) // 2", "half = M + 1", "reconstruction not balanced"),
    ("bt = \"T\" if transb.upper() == \"N\" else \"N\"", "bt = transb.upper()",
     "op(B) transposed"),
    ("v = a * X[i, j] * Fraction(2) ** int(ea[i] + eb[j] - 2 * p)",
     "v = a * X[i, j] * Fraction(2) ** int(ea[i] + eb[j] - p)", "wrong result scale"),
    ("v += b * (Fraction(ch[i + j * ldc]) + Fraction(cl[i + j * ldc]))",
     "v += b * Fraction(ch[i + j * ldc])", "low part of C dropped"),
    ("im.append(t3 - t1 - t2)", "im.append(t3 - t1 + t2)", "three-product sign"),
    ("return scale_exponents(np.concatenate([rh, ih], axis=1))", "return scale_exponents(rh)",
     "complex exponent from the real part only"),
    ("p = exponent(k, count, margin_bits=3)", "p = exponent(k, count)",
     "complex margin too small"),
    ("    if trans.upper() == \"C\":\n        ih, il = -ih, -il", "    if False:\n        ih, il = -ih, -il",
     "conjugation of op(A) lost"),
    ("bt = {\"N\": \"T\", \"T\": \"N\", \"C\": \"C\"}[transb.upper()]",
     "bt = {\"N\": \"T\", \"T\": \"N\", \"C\": \"N\"}[transb.upper()]",
     "conjugation of op(B) lost"),
    ("vr, vi = ar * pr - ai * pi, ar * pi + ai * pr", "vr, vi = ar * pr + ai * pi, ar * pi + ai * pr",
     "complex alpha sign"),
    ("            t = t - np.ldexp(c, QD_CHUNK_BITS * j)",
     "            t = t - np.ldexp(c, QD_CHUNK_BITS * j - 1)", "qd chunk removed at the wrong weight"),
    ("    for x in parts:\n        t = np.rint", "    for x in parts[:3]:\n        t = np.rint",
     "qd last part dropped"),
    ("(mid - hi - lo) * (1 << QD_SPLIT_BITS)", "(mid - hi + lo) * (1 << QD_SPLIT_BITS)",
     "qd three-product sign"),
    ("return modulus_product(count).bit_length() - 1 >= 215 + lk",
     "return modulus_product(count).bit_length() - 1 >= 205 + lk", "qd moduli margin"),
    ("    x1 = sum(obj[j] * (1 << (QD_CHUNK_BITS * (j - 4))) for j in range(4, 8))",
     "    x1 = sum(obj[j] * (1 << (QD_CHUNK_BITS * (j - 3))) for j in range(4, 8))",
     "qd high half misplaced"),
]

CHECKS = [("moduli", lambda c, r: check_moduli(c)),
          ("exponent", lambda c, r: check_exponent(c)),
          ("integers", check_integers),
          ("residues", check_residues),
          ("reconstruct", lambda c, r: check_reconstruct(c)),
          ("integer_product", check_integer_product),
          ("rgemm", check_rgemm),
          ("complex_exponents", lambda c, r: check_complex_exponents(c)),
          ("complex_integer_product", check_complex_integer_product),
          ("cgemm", check_cgemm),
          ("qd_split", check_qd_split),
          ("qd_count", lambda c, r: check_qd_count(c)),
          ("qd_integer_product", check_qd_integer_product),
          ("qgemm", check_qgemm)]


def _load_copy(text, tmp):
    path = os.path.join(tmp, "crt_mutant.py")
    with open(path, "w") as f:
        f.write(text)
    spec = importlib.util.spec_from_file_location("crt_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _caught(mod):
    for name, check in CHECKS:
        try:
            check(mod, np.random.default_rng(21))
        except Exception:
            return name
    return None


@pytest.mark.parametrize("orig,mut,what", MUTANTS, ids=[m[2] for m in MUTANTS])
def test_crt_mutant_is_caught(orig, mut, what):
    src = open(CRT.__file__).read()
    assert src.count(orig) == 1, what
    with tempfile.TemporaryDirectory() as tmp:
        mod = _load_copy(src.replace(orig, mut), tmp)
        assert _caught(mod) is not None, what


def test_crt_unmutated_copy_passes():
    with tempfile.TemporaryDirectory() as tmp:
        mod = _load_copy(open(CRT.__file__).read(), tmp)
        assert _caught(mod) is None

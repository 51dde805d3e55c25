"""Pins of the CPU oracle against facts that do not come from the oracle.

Each check takes a loaded oracle library (the real one, or a deliberately
broken copy in test_oracle_mutants.py) and raises AssertionError when the
library disagrees with:

* the manual's worked Rgemm example (tests/golden/rgemm_worked_example.txt);
* exact rational arithmetic (fractions.Fraction) on small random dd inputs,
  within the first-order error bound of the dd algorithms;
* BLAS argument-position error codes (tests/golden/blas_arg_positions.txt);
* algebraic identities that hold bit-exactly (identity matrices, alpha = 0,
  beta = 0 with NaN C, quick returns, transposed copies, Rsyrk vs Rgemm,
  untouched padding and opposite triangle);
* exact digit reconstruction and exact slice products of the split form.
"""
import os
from fractions import Fraction

import numpy as np

import oracle
import workloads as W
from oracle.compare import bits

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U2 = Fraction(1, 2 ** 106)          # u^2, u = 2^-53


def F(h, l=0.0):
    return Fraction(float(h)) + Fraction(float(l))


def read_worked_example():
    vals = {"A": [], "B": [], "C": [], "ANSWER": []}
    alpha = beta = None
    with open(os.path.join(GOLDEN, "rgemm_worked_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            if key == "alpha":
                alpha = float(rest[0])
            elif key == "beta":
                beta = float(rest[0])
            else:
                vals[key].append([float(x) for x in rest])
    return alpha, beta, {k: np.array(v) for k, v in vals.items()}


def read_arg_positions():
    out = {}
    with open(os.path.join(GOLDEN, "blas_arg_positions.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                r, a, p = line.split()
                out[(r, a)] = int(p)
    return out


def colmajor(M):
    return np.asfortranarray(M).flatten(order="F").copy()


# ---- worked example -------------------------------------------------------------

def check_worked_example(lib):
    alpha, beta, v = read_worked_example()
    z = np.zeros(9)
    for ta in "NT":
        for tb in "NT":
            A = v["A"] if ta == "N" else v["A"].T
            B = v["B"] if tb == "N" else v["B"].T
            Ch, Cl = colmajor(v["C"]), z.copy()
            info = oracle.rgemm(ta, tb, 3, 3, 3, alpha, (colmajor(A), z.copy()), 3,
                                (colmajor(B), z.copy()), 3, beta, (Ch, Cl), 3, lib=lib)
            assert info == 0
            assert np.array_equal(Ch, colmajor(v["ANSWER"])), (ta, tb, Ch)
            assert np.all(Cl == 0.0)


# ---- exact rational brute force -----------------------------------------------------

def exact_entry(case, i, j, opA, opB):
    k = case["k"]
    s = sum((opA(i, l) * opB(l, j) for l in range(k)), Fraction(0))
    return s


def _op(flat_h, flat_l, ld, trans):
    def f(r, c):
        idx = (c + r * ld) if trans else (r + c * ld)
        return F(flat_h[idx], flat_l[idx])
    return f


def _abs_op(flat_h, flat_l, ld, trans):
    g = _op(flat_h, flat_l, ld, trans)
    return lambda r, c: abs(g(r, c))


def gemm_bound(k):
    """First-order bound of the oracle's evaluation, in units of
    (|alpha| sum_l |a_il b_lj| + |beta c_ij|): per product 4u^2 (DWTimesDW3),
    per accumulation 3u^2 (AccurateDWPlusDW), then the alpha and beta
    products and the final add, plus slack for second-order terms."""
    return (3 * k + 12) * U2 * Fraction(101, 100)


def check_exact_gemm(lib, seeds=range(6), dist="uniform", sizes=None):
    sizes = sizes or [(1, 1, 1), (2, 3, 4), (5, 4, 6), (6, 6, 6), (3, 5, 1), (4, 1, 5)]
    for seed in seeds:
        for (m, n, k) in sizes:
            for ta in "NT":
                for tb in "NT":
                    c = W.gemm_case(1000 + seed, ta, tb, m, n, k, dist=dist)
                    C0h, C0l = c["C"][0].copy(), c["C"][1].copy()
                    info = oracle.rgemm(ta, tb, m, n, k, c["alpha"], c["A"], c["lda"], c["B"],
                                        c["ldb"], c["beta"], c["C"], c["ldc"], lib=lib)
                    assert info == 0
                    opA = _op(*c["A"], c["lda"], ta == "T")
                    opB = _op(*c["B"], c["ldb"], tb == "T")
                    al, be = F(*c["alpha"]), F(*c["beta"])
                    bnd = gemm_bound(k)
                    for i in range(m):
                        for j in range(n):
                            idx = i + j * c["ldc"]
                            c0 = F(C0h[idx], C0l[idx])
                            dot = exact_entry(c, i, j, opA, opB)
                            absdot = sum((abs(opA(i, l) * opB(l, j)) for l in range(k)),
                                         Fraction(0))
                            exact = al * dot + be * c0
                            got = F(c["C"][0][idx], c["C"][1][idx])
                            tol = bnd * (abs(al) * absdot + abs(be) * abs(c0))
                            assert abs(got - exact) <= tol, (seed, m, n, k, ta, tb, i, j,
                                                             float(abs(got - exact)), float(tol))
                            # normalised output: hi + lo rounds to hi
                            assert c["C"][0][idx] + c["C"][1][idx] == c["C"][0][idx]
                    # padding rows untouched
                    ldc = c["ldc"]
                    pad = np.ones(ldc * n, bool)
                    for j in range(n):
                        pad[j * ldc: j * ldc + m] = False
                    assert np.array_equal(bits(c["C"][0])[pad], bits(C0h)[pad])
                    assert np.array_equal(bits(c["C"][1])[pad], bits(C0l)[pad])


def check_exact_syrk(lib, seeds=range(4), dist="uniform"):
    for seed in seeds:
        for (n, k) in [(1, 1), (3, 2), (5, 6), (6, 4), (4, 1)]:
            for uplo in "UL":
                for trans in "NT":
                    c = W.syrk_case(2000 + seed, uplo, trans, n, k, dist=dist)
                    C0h, C0l = c["C"][0].copy(), c["C"][1].copy()
                    info = oracle.rsyrk(uplo, trans, n, k, c["alpha"], c["A"], c["lda"],
                                        c["beta"], c["C"], c["ldc"], lib=lib)
                    assert info == 0
                    opA = _op(*c["A"], c["lda"], trans == "T")
                    opB = _op(*c["A"], c["lda"], trans == "N")
                    al, be = F(*c["alpha"]), F(*c["beta"])
                    bnd = gemm_bound(k)
                    ldc = c["ldc"]
                    for j in range(n):
                        for i in range(n):
                            idx = i + j * ldc
                            inside = (i <= j) if uplo == "U" else (i >= j)
                            if not inside:
                                assert bits(c["C"][0][idx:idx + 1])[0] == bits(C0h[idx:idx + 1])[0]
                                assert bits(c["C"][1][idx:idx + 1])[0] == bits(C0l[idx:idx + 1])[0]
                                continue
                            c0 = F(C0h[idx], C0l[idx])
                            dot = sum((opA(i, l) * opB(l, j) for l in range(k)), Fraction(0))
                            absdot = sum((abs(opA(i, l) * opB(l, j)) for l in range(k)),
                                         Fraction(0))
                            exact = al * dot + be * c0
                            got = F(c["C"][0][idx], c["C"][1][idx])
                            tol = bnd * (abs(al) * absdot + abs(be) * abs(c0))
                            assert abs(got - exact) <= tol, (seed, n, k, uplo, trans, i, j)


# ---- argument checking ------------------------------------------------------------

def gemm_info(lib, transa="N", transb="N", m=2, n=2, k=2, lda=None, ldb=None, ldc=None):
    nra = m if transa.upper() == "N" else k
    nrb = k if transb.upper() == "N" else n
    lda = max(1, nra) if lda is None else lda
    ldb = max(1, nrb) if ldb is None else ldb
    ldc = max(1, m) if ldc is None else ldc
    buf = np.full(64, np.nan)
    sent = buf.copy()
    info = oracle.rgemm(transa, transb, m, n, k, (1.0, 0.0), (buf, buf), lda, (buf, buf), ldb,
                        (0.5, 0.0), (sent, sent), ldc, lib=lib)
    return info, sent


def syrk_info(lib, uplo="U", trans="N", n=2, k=2, lda=None, ldc=None):
    nra = n if trans.upper() == "N" else k
    lda = max(1, nra) if lda is None else lda
    ldc = max(1, n) if ldc is None else ldc
    buf = np.full(64, np.nan)
    sent = buf.copy()
    info = oracle.rsyrk(uplo, trans, n, k, (1.0, 0.0), (buf, buf), lda, (0.5, 0.0),
                        (sent, sent), ldc, lib=lib)
    return info, sent


def check_info_codes(lib):
    pos = read_arg_positions()
    g = lambda **kw: gemm_info(lib, **kw)[0]
    s = lambda **kw: syrk_info(lib, **kw)[0]
    assert g() == 0
    for ta in "NnTtCc":
        assert g(transa=ta) == 0 and g(transb=ta) == 0
    assert g(transa="X") == pos[("gemm", "transa")]
    assert g(transb="q") == pos[("gemm", "transb")]
    assert g(transa="X", m=-1) == pos[("gemm", "transa")]          # first bad one wins
    assert g(m=-1) == pos[("gemm", "m")]
    assert g(n=-1) == pos[("gemm", "n")]
    assert g(k=-1) == pos[("gemm", "k")]
    assert g(m=5, lda=4) == pos[("gemm", "lda")]
    assert g(transa="T", m=5, k=3, lda=3) == 0
    assert g(transa="T", m=3, k=5, lda=4) == pos[("gemm", "lda")]
    assert g(k=5, ldb=4) == pos[("gemm", "ldb")]
    assert g(transb="T", n=5, k=3, ldb=4) == pos[("gemm", "ldb")]
    assert g(transb="T", n=3, k=5, ldb=3) == 0
    assert g(m=5, lda=5, ldc=4) == pos[("gemm", "ldc")]
    assert g(m=0, lda=0) == pos[("gemm", "lda")]                   # ld >= max(1, rows)
    assert g(m=0, lda=1, ldc=1) == 0
    assert s() == 0
    assert s(uplo="x") == pos[("syrk", "uplo")]
    assert s(trans="z") == pos[("syrk", "trans")]
    assert s(trans="c") == 0
    assert s(n=-1) == pos[("syrk", "n")]
    assert s(k=-1) == pos[("syrk", "k")]
    assert s(n=5, lda=4) == pos[("syrk", "lda")]
    assert s(trans="T", n=5, k=3, lda=3) == 0
    assert s(trans="T", n=3, k=5, lda=4) == pos[("syrk", "lda")]
    assert s(n=5, lda=5, ldc=4) == pos[("syrk", "ldc")]
    # an invalid call writes nothing
    info, sent = gemm_info(lib, m=-1)
    assert info and np.all(np.isnan(sent))


# ---- identities -------------------------------------------------------------------

def _eye(n, ld):
    h = np.zeros(ld * n)
    for i in range(n):
        h[i + i * ld] = 1.0
    return h, np.zeros(ld * n)


def check_identities(lib):
    rng = W.streams(77)
    m, n, k = 7, 5, 6
    # I * B = B and A * I = A, bit-exact
    c = W.gemm_case(3001, "N", "N", k, n, k)
    I = _eye(k, c["lda"])
    C = (np.full(c["ldc"] * n, np.nan), np.full(c["ldc"] * n, np.nan))
    assert oracle.rgemm("N", "N", k, n, k, (1.0, 0.0), I, c["lda"], c["B"], c["ldb"], (0.0, 0.0),
                        C, c["ldc"], lib=lib) == 0
    for j in range(n):
        sl = slice(j * c["ldc"], j * c["ldc"] + k)
        bl = slice(j * c["ldb"], j * c["ldb"] + k)
        assert np.array_equal(C[0][sl], c["B"][0][bl]) and np.array_equal(C[1][sl], c["B"][1][bl])
    c = W.gemm_case(3002, "N", "N", m, k, k)
    I = _eye(k, c["ldb"])
    C = (np.full(c["ldc"] * k, np.nan), np.full(c["ldc"] * k, np.nan))
    assert oracle.rgemm("N", "N", m, k, k, (1.0, 0.0), c["A"], c["lda"], I, c["ldb"], (0.0, 0.0),
                        C, c["ldc"], lib=lib) == 0
    for j in range(k):
        sl = slice(j * c["ldc"], j * c["ldc"] + m)
        al = slice(j * c["lda"], j * c["lda"] + m)
        assert np.array_equal(C[0][sl], c["A"][0][al]) and np.array_equal(C[1][sl], c["A"][1][al])

    # beta = 0: C is never read (NaN in, finite out); alpha = 0 and beta = 0: +0
    c = W.gemm_case(3003, "N", "T", m, n, k, c_nan=True, beta_zero=True)
    assert oracle.rgemm("N", "T", m, n, k, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"],
                        (0.0, 0.0), c["C"], c["ldc"], lib=lib) == 0
    for j in range(n):
        assert np.all(np.isfinite(c["C"][0][j * c["ldc"]: j * c["ldc"] + m]))
    c = W.gemm_case(3004, "T", "N", m, n, k, c_nan=True)
    assert oracle.rgemm("T", "N", m, n, k, (0.0, 0.0), (None, None), c["lda"], (None, None),
                        c["ldb"], (0.0, 0.0), c["C"], c["ldc"], lib=lib) == 0
    for j in range(n):
        col = slice(j * c["ldc"], j * c["ldc"] + m)
        assert np.all(bits(c["C"][0][col]) == 0) and np.all(bits(c["C"][1][col]) == 0)

    # alpha = 0 (A, B not read) and k = 0: C = beta * C within the dd-mul bound
    for kk, al in ((k, (0.0, 0.0)), (0, (0.75, 0.0))):
        c = W.gemm_case(3005 + kk, "N", "N", m, n, max(kk, 1))
        C0 = (c["C"][0].copy(), c["C"][1].copy())
        assert oracle.rgemm("N", "N", m, n, kk, al, (None, None), c["lda"], (None, None),
                            c["ldb"], c["beta"], c["C"], c["ldc"], lib=lib) == 0
        be = F(*c["beta"])
        for j in range(n):
            for i in range(m):
                idx = i + j * c["ldc"]
                exact = be * F(C0[0][idx], C0[1][idx])
                got = F(c["C"][0][idx], c["C"][1][idx])
                assert abs(got - exact) <= 5 * U2 * abs(exact)

    # quick returns leave C bit-identical (NaN payloads included)
    for args in ((0, n, k, c["alpha"], c["beta"]), (m, 0, k, c["alpha"], c["beta"]),
                 (m, n, k, (0.0, 0.0), (1.0, 0.0)), (m, n, 0, c["alpha"], (1.0, 0.0))):
        cc = W.gemm_case(3010, "N", "N", m, n, k, c_nan=True)
        before = (bits(cc["C"][0]).copy(), bits(cc["C"][1]).copy())
        mm, nn, kk, al, be = args
        assert oracle.rgemm("N", "N", mm, nn, kk, al, cc["A"], cc["lda"], cc["B"], cc["ldb"], be,
                            cc["C"], cc["ldc"], lib=lib) == 0
        assert np.array_equal(bits(cc["C"][0]), before[0])
        assert np.array_equal(bits(cc["C"][1]), before[1])

    # transposed copies give bit-identical results through all four op forms
    c = W.gemm_case(3020, "N", "N", m, n, k, padded=False)
    Ah = c["A"][0][: m * k].reshape(k, m).T
    Al = c["A"][1][: m * k].reshape(k, m).T
    Bh = c["B"][0][: k * n].reshape(n, k).T
    Bl = c["B"][1][: k * n].reshape(n, k).T
    ref = None
    for ta in "NT":
        for tb in "NT":
            A = (colmajor(Ah if ta == "N" else Ah.T), colmajor(Al if ta == "N" else Al.T))
            B = (colmajor(Bh if tb == "N" else Bh.T), colmajor(Bl if tb == "N" else Bl.T))
            C = (c["C"][0].copy(), c["C"][1].copy())
            assert oracle.rgemm(ta, tb, m, n, k, c["alpha"], A, m if ta == "N" else k, B,
                                k if tb == "N" else n, c["beta"], C, m, lib=lib) == 0
            if ref is None:
                ref = C
            else:
                assert np.array_equal(bits(C[0]), bits(ref[0])), (ta, tb)
                assert np.array_equal(bits(C[1]), bits(ref[1])), (ta, tb)

    # Rsyrk equals Rgemm(op(A), op(A)^T) bit-for-bit on its triangle
    for uplo in "UL":
        for trans in "NT":
            s = W.syrk_case(3030, uplo, trans, 9, 4)
            C0 = (s["C"][0].copy(), s["C"][1].copy())
            G = (s["C"][0].copy(), s["C"][1].copy())
            assert oracle.rsyrk(uplo, trans, 9, 4, s["alpha"], s["A"], s["lda"], s["beta"],
                                s["C"], s["ldc"], lib=lib) == 0
            tb = "T" if trans == "N" else "N"
            assert oracle.rgemm(trans, tb, 9, 9, 4, s["alpha"], s["A"], s["lda"], s["A"], s["lda"],
                                s["beta"], G, s["ldc"], lib=lib) == 0
            for j in range(9):
                for i in range(9):
                    idx = i + j * s["ldc"]
                    inside = (i <= j) if uplo == "U" else (i >= j)
                    want = (G[0][idx], G[1][idx]) if inside else (C0[0][idx], C0[1][idx])
                    assert bits(np.array([s["C"][0][idx]]))[0] == bits(np.array([want[0]]))[0]
                    assert bits(np.array([s["C"][1][idx]]))[0] == bits(np.array([want[1]]))[0]

    # integer data with small partial sums: bit-exact integers
    ri = W.streams(3040)
    m2, n2, k2 = 9, 8, 11
    A = W.dd_matrix(ri[0], m2, k2, dist="int")
    B = W.dd_matrix(ri[1], k2, n2, dist="int")
    C = W.dd_matrix(ri[2], m2, n2, dist="int")
    want = 3 * (A[0].reshape(k2, m2).T @ B[0].reshape(n2, k2).T) - 2 * C[0].reshape(n2, m2).T
    assert oracle.rgemm("N", "N", m2, n2, k2, (3.0, 0.0), A, m2, B, k2, (-2.0, 0.0), C, m2,
                        lib=lib) == 0
    assert np.array_equal(C[0].reshape(n2, m2).T, want) and np.all(C[1] == 0.0)


# ---- split form -----------------------------------------------------------------------

def _split_forms(k, nslices):
    """(wfirst, w, qmax) of every digit form the split oracle serves: INT8 with
    8-bit and with 7-bit later digits (carried into int8's range), FP64."""
    return [(6, 8, oracle.INT8_QMAX), (6, 7, oracle.INT8_QMAX),
            oracle.fp64_digit_width(k, nslices) + (0,)]


def check_ozaki_split_exact(lib, dist="wide", nslices=18):
    """Digits reconstruct the scaled value exactly up to the last remainder,
    stay within their bounds, and the scale puts every row inside (-1, 1);
    a digit after the first that would exceed int8's range is carried into
    the digit before it (checked on inputs whose digits are worked out by
    hand)."""
    for (rows, k, trans) in [(5, 7, False), (4, 9, True), (1, 1, False)]:
        rng = W.streams(4000 + rows)[0]
        ld = rows + 2 if not trans else k + 1
        nr, nc = (rows, k) if not trans else (k, rows)
        X = W.dd_matrix(rng, nr, nc, ld, dist=dist)
        sr, sl = (1, ld) if not trans else (ld, 1)
        for (wf, w, qmax) in _split_forms(k, nslices):
            # digits may carry only where the rounded range [-2^(w-1), 2^(w-1)]
            # exceeds qmax
            carries = qmax > 0 and 2 ** (w - 1) > qmax
            exps, digs = oracle.ozaki_split(rows, k, X, sr, sl, nslices, wf, w, qmax, lib=lib)
            for r in range(rows):
                vals = [F(X[0][r * sr + l * sl], X[1][r * sr + l * sl]) for l in range(k)]
                mx = max(abs(float(X[0][r * sr + l * sl])) for l in range(k))
                e = int(exps[r])
                assert Fraction(2) ** (e - 1) <= Fraction(mx) < Fraction(2) ** e
                for l in range(k):
                    x = vals[l] / Fraction(2) ** e
                    assert abs(x) < 1
                    recon = Fraction(0)
                    for t in range(nslices):
                        q = int(digs[t, r, l])
                        if t == 0:
                            assert abs(q) <= 2 ** wf + (1 if carries else 0), (t, q)
                        else:
                            assert -2 ** (w - 1) <= q <= 2 ** (w - 1), (t, q)
                            if qmax > 0:
                                assert q <= qmax, (t, q, qmax)
                        W_t = wf + w * t
                        recon += Fraction(q, 2 ** W_t)
                        # remainder after digit t lies within half a unit of
                        # it, plus the unit a carry from digit t+1 may add
                        slack = 1 if (carries and t < nslices - 1) else 0
                        assert abs(x - recon) <= (Fraction(1, 2) + slack) / 2 ** W_t * Fraction(
                            1000001, 1000000), (t, float(x - recon))
    # worked carries (first digit width 6, later 8, int8 storage): a row
    # [0.75, x] has scale exponent 0, so x's digits are those of x itself.
    #   x = (20 + 127.75/256) / 64: rounded digits 20, 128 (127.75 rounds
    #   up), -64 (the remainder -0.25 times 256), then 0; 128 exceeds 127,
    #   so it becomes 128 - 256 = -128 and the first digit 21.
    #   x = (20 + (127 + 127.75/256)/256) / 64: rounded digits 20, 127, 128,
    #   -64; the carry out of the third digit makes the second 128, which
    #   carries again: 21, -128, -128, -64.
    cases = [(Fraction(20 * 256 + Fraction(511, 4), 256 * 64), [21, -128, -64, 0, 0]),
             (Fraction(20 * 256 * 256 + 127 * 256 + Fraction(511, 4), 256 * 256 * 64),
              [21, -128, -128, -64, 0])]
    for x, want in cases:
        hi = float(x)
        lo = float(x - Fraction(hi))
        X = (np.array([0.75, hi]), np.array([0.0, lo]))
        exps, digs = oracle.ozaki_split(1, 2, X, 0, 1, 5, 6, 8, oracle.INT8_QMAX, lib=lib)
        assert int(exps[0]) == 0
        assert [int(v) for v in digs[:, 0, 1]] == want, (digs[:, 0, 1], want)
        recon = sum(Fraction(int(q), 2 ** (6 + 8 * t)) for t, q in enumerate(digs[:, 0, 1]))
        assert recon == x
        # without the storage limit the rounded digits stay as they are
        _, raw = oracle.ozaki_split(1, 2, X, 0, 1, 5, 6, 8, 0, lib=lib)
        assert int(raw[0, 0, 1]) == 20 and 128 in [int(v) for v in raw[:, 0, 1]]


def check_ozaki_gemm_exact(lib):
    """Split-form result vs exact rational arithmetic on the same digits: the
    recombination of the kept anti-diagonals must match the exact sum of the
    kept digit products to within the dd rounding of the final steps."""
    m, n, k, s = 4, 3, 5, 6
    for ta in "NT":
        for tb in "NT":
            c = W.gemm_case(5000, ta, tb, m, n, k, dist="wide")
            for (wf, w, qmax) in _split_forms(k, s):
                C = (c["C"][0].copy(), c["C"][1].copy())
                C0 = (c["C"][0].copy(), c["C"][1].copy())
                assert oracle.ozaki_rgemm(ta, tb, m, n, k, c["alpha"], c["A"], c["lda"], c["B"],
                                          c["ldb"], c["beta"], C, c["ldc"], s, wf, w, qmax,
                                          lib=lib) == 0
                ea, qa = oracle.ozaki_split(m, k, c["A"], c["lda"] if ta == "T" else 1,
                                            1 if ta == "T" else c["lda"], s, wf, w, qmax,
                                            lib=lib)
                eb, qb = oracle.ozaki_split(n, k, c["B"], 1 if tb == "T" else c["ldb"],
                                            c["ldb"] if tb == "T" else 1, s, wf, w, qmax,
                                            lib=lib)
                al, be = F(*c["alpha"]), F(*c["beta"])
                for i in range(m):
                    for j in range(n):
                        p = Fraction(0)
                        for t in range(1, s + 1):
                            for u in range(1, s + 2 - t):
                                x = sum(int(qa[t - 1, i, l]) * int(qb[u - 1, j, l])
                                        for l in range(k))
                                p += Fraction(x, 2 ** (2 * wf + w * (t + u - 2)))
                        p *= Fraction(2) ** (int(ea[i]) + int(eb[j]))
                        idx = i + j * c["ldc"]
                        c0 = F(C0[0][idx], C0[1][idx])
                        exact = al * p + be * c0
                        got = F(C[0][idx], C[1][idx])
                        tol = (2 * (s + 1) + 12) * U2 * (abs(al * p) + abs(be * c0)) * 2
                        assert abs(got - exact) <= tol, (ta, tb, i, j, wf, w)


# ---- primitives --------------------------------------------------------------------

def check_primitives(lib, count=400):
    rng = np.random.Generator(np.random.PCG64(6000))
    a = rng.uniform(-1, 1, count) * np.ldexp(1.0, rng.integers(-60, 60, count))
    b = rng.uniform(-1, 1, count) * np.ldexp(1.0, rng.integers(-60, 60, count))
    for x, y in zip(a, b):
        s, e = oracle.two_sum(x, y, lib=lib)
        assert F(s) + F(e) == F(x) + F(y) and s == x + y
        p, e = oracle.two_prod(x, y, lib=lib)
        assert F(p) + F(e) == F(x) * F(y) and p == x * y
    xs = W.dd_values(rng, count, "wide")
    ys = W.dd_values(rng, count, "wide")
    for t in range(count):
        x = (xs[0][t], xs[1][t])
        y = (ys[0][t], ys[1][t])
        z = oracle.dd_add(x, y, lib=lib)
        ex = F(*x) + F(*y)
        assert abs(F(*z) - ex) <= (3 * U2 + 13 * U2 / 2 ** 53) * abs(ex)
        assert z[0] + z[1] == z[0]
        z = oracle.dd_mul(x, y, lib=lib)
        ex = F(*x) * F(*y)
        assert abs(F(*z) - ex) <= 4 * U2 * abs(ex)
        assert z[0] + z[1] == z[0]
    # heavy cancellation: y.hi = -x.hi (or one ulp away); the accurate add's
    # relative bound must still hold, which a sloppy add misses
    for t in range(count):
        x = (xs[0][t], xs[1][t])
        yh = -x[0] if t % 2 else -np.nextafter(x[0], 0.0)
        yl = ys[1][t] * 2.0 ** float(np.floor(np.log2(abs(x[0]) + 1e-300)) -
                                     np.floor(np.log2(abs(ys[0][t]))))
        y = oracle.two_sum(yh, yl, lib=lib)
        z = oracle.dd_add(x, y, lib=lib)
        ex = F(*x) + F(*y)
        assert abs(F(*z) - ex) <= (3 * U2 + 13 * U2 / 2 ** 53) * abs(ex), (t, x, y)


# ---- complex dd Cgemm ----------------------------------------------------------------

def read_cgemm_example():
    """The manual's Cgemm demo as decimal strings: dict with alpha, beta ((re, im)
    strings) and A, B, C, ANSWER_BINARY64, ANSWER_DECIMAL (3 x 3 lists of
    (re, im) strings, row by row)."""
    out = {"A": [], "B": [], "C": [], "ANSWER_BINARY64": [], "ANSWER_DECIMAL": []}
    with open(os.path.join(GOLDEN, "cgemm_worked_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, rest = line.split(None, 1)
            ents = [tuple(e.split()) for e in rest.split("|")]
            if key in ("alpha", "beta"):
                out[key] = ents[0]
            else:
                out[key].append(ents)
    return out


def _dd_of(x):
    """Nearest dd (hi, lo) of an exact rational."""
    hi = float(x)
    return hi, float(x - Fraction(hi))


def _cplanes(rows, conv):
    """3 x 3 (re, im) entries -> four column-major planes through conv(str) -> (hi, lo)."""
    n = len(rows)
    planes = [np.zeros(n * n) for _ in range(4)]
    for i in range(n):
        for j in range(n):
            (rh, rl), (ih, il) = conv(rows[i][j][0]), conv(rows[i][j][1])
            for p, v in zip(planes, (rh, rl, ih, il)):
                p[i + j * n] = v
    return tuple(planes)


def _exact_cgemm(alpha, A, B, beta, C):
    """alpha A B + beta C over the rationals; entries complex as (re, im) Fractions."""
    n = len(A)

    def mul(x, y):
        return (x[0] * y[0] - x[1] * y[1], x[0] * y[1] + x[1] * y[0])

    out = []
    for i in range(n):
        row = []
        for j in range(n):
            acc = (Fraction(0), Fraction(0))
            for l in range(n):
                p = mul(A[i][l], B[l][j])
                acc = (acc[0] + p[0], acc[1] + p[1])
            a, b = mul(alpha, acc), mul(beta, C[i][j])
            row.append((a[0] + b[0], a[1] + b[1]))
        out.append(row)
    return out


def cgemm_bound(k):
    """Per-component first-order bound of the dd Cgemm evaluation in units of
    (|alpha|_1 sum_l |a_il|_1 |b_lj|_1 + |beta|_1 |c_ij|_1), |z|_1 = |re| + |im|:
    each complex product is two dd products and a dd add (7 u^2), each of the k
    running sums adds 3 u^2, and alpha, beta and the final add another 17 u^2."""
    return (3 * k + 24) * U2 * Fraction(101, 100)


def _abs1(z):
    return abs(z[0]) + abs(z[1])


def check_cgemm_worked_example(lib):
    ex = read_cgemm_example()
    dec = lambda s: Fraction(s)                     # noqa: E731
    b64 = lambda s: Fraction(float(s))              # noqa: E731
    for conv, ans_key, inflate in ((b64, "ANSWER_BINARY64", 0), (dec, "ANSWER_DECIMAL", 6)):
        A = [[(conv(r), conv(i)) for r, i in row] for row in ex["A"]]
        B = [[(conv(r), conv(i)) for r, i in row] for row in ex["B"]]
        C = [[(conv(r), conv(i)) for r, i in row] for row in ex["C"]]
        al = (conv(ex["alpha"][0]), conv(ex["alpha"][1]))
        be = (conv(ex["beta"][0]), conv(ex["beta"][1]))
        exact = _exact_cgemm(al, A, B, be, C)
        printed = [[(Fraction(r), Fraction(i)) for r, i in row] for row in ex[ans_key]]
        # the fixture itself: the printed answer is the exact result (the decimal
        # one exactly, the 64-digit one to its printed digits)
        for i in range(3):
            for j in range(3):
                for c in range(2):
                    d = abs(printed[i][j][c] - exact[i][j][c])
                    assert d <= Fraction(1, 10 ** 60) * max(abs(exact[i][j][c]), 1), (ans_key, i, j)
        # the oracle on the dd-rounded inputs (binary64 inputs are exact dd numbers)
        todd = lambda s: _dd_of(conv(s))            # noqa: E731
        Ap, Bp, Cp = _cplanes(ex["A"], todd), _cplanes(ex["B"], todd), _cplanes(ex["C"], todd)
        alpha = (todd(ex["alpha"][0]), todd(ex["alpha"][1]))
        beta = (todd(ex["beta"][0]), todd(ex["beta"][1]))
        bnd = cgemm_bound(3) + inflate * U2
        for ta, tb in W.COPS:
            # op(X) of the transformed copy is X itself
            def prep(P, t):
                M = [p.reshape(3, 3, order="F") for p in P]
                if t != "N":
                    M = [m.T for m in M]
                if t == "C":
                    M[2], M[3] = -M[2], -M[3]
                return tuple(colmajor(m) for m in M)
            Cw = tuple(p.copy() for p in Cp)
            info = oracle.cgemm(ta, tb, 3, 3, 3, alpha, prep(Ap, ta), 3, prep(Bp, tb), 3, beta, Cw,
                                3, lib=lib)
            assert info == 0
            for i in range(3):
                for j in range(3):
                    idx = i + 3 * j
                    scale = _abs1(al) * sum(_abs1(A[i][l]) * _abs1(B[l][j]) for l in range(3)) \
                        + _abs1(be) * _abs1(C[i][j])
                    got = (F(Cw[0][idx], Cw[1][idx]), F(Cw[2][idx], Cw[3][idx]))
                    for c in range(2):
                        err = abs(got[c] - printed[i][j][c])
                        assert err <= bnd * scale + Fraction(1, 10 ** 60) * scale, (
                            ans_key, ta, tb, i, j, c, float(err / scale))


def _cop(planes, ld, t):
    """op(X)(r, c) as an exact (re, im) pair of Fractions; t in N, T, C."""
    rh, rl, ih, il = planes

    def get(r, c):
        idx = (c + r * ld) if t != "N" else (r + c * ld)
        re, im = F(rh[idx], rl[idx]), F(ih[idx], il[idx])
        return (re, -im) if t == "C" else (re, im)
    return get


def check_exact_cgemm(lib, seeds=range(2), dist="uniform",
                      sizes=((1, 1, 1), (2, 3, 4), (4, 3, 2), (3, 1, 5))):
    for seed in seeds:
        for (m, n, k) in sizes:
            for ta, tb in W.COPS:
                c = W.cgemm_case(3000 + seed, ta, tb, m, n, k, dist=dist)
                C0 = tuple(p.copy() for p in c["C"])
                info = oracle.cgemm(ta, tb, m, n, k, c["alpha"], c["A"], c["lda"], c["B"],
                                    c["ldb"], c["beta"], c["C"], c["ldc"], lib=lib)
                assert info == 0
                opA, opB = _cop(c["A"], c["lda"], ta), _cop(c["B"], c["ldb"], tb)
                al = (F(*c["alpha"][0]), F(*c["alpha"][1]))
                be = (F(*c["beta"][0]), F(*c["beta"][1]))
                bnd = cgemm_bound(k)
                for i in range(m):
                    for j in range(n):
                        idx = i + j * c["ldc"]
                        c0 = (F(C0[0][idx], C0[1][idx]), F(C0[2][idx], C0[3][idx]))
                        acc = [Fraction(0), Fraction(0)]
                        mag = Fraction(0)
                        for l in range(k):
                            a, b = opA(i, l), opB(l, j)
                            acc[0] += a[0] * b[0] - a[1] * b[1]
                            acc[1] += a[0] * b[1] + a[1] * b[0]
                            mag += _abs1(a) * _abs1(b)
                        ex = (al[0] * acc[0] - al[1] * acc[1] + be[0] * c0[0] - be[1] * c0[1],
                              al[0] * acc[1] + al[1] * acc[0] + be[0] * c0[1] + be[1] * c0[0])
                        tol = bnd * (_abs1(al) * mag + _abs1(be) * _abs1(c0))
                        got = (F(c["C"][0][idx], c["C"][1][idx]), F(c["C"][2][idx], c["C"][3][idx]))
                        for q in range(2):
                            assert abs(got[q] - ex[q]) <= tol, (seed, m, n, k, ta, tb, i, j, q)
                            h = c["C"][2 * q][idx]
                            assert h + c["C"][2 * q + 1][idx] == h      # normalised
                # padding rows of every plane untouched
                ldc = c["ldc"]
                pad = np.ones(ldc * n, bool)
                for j in range(n):
                    pad[j * ldc: j * ldc + m] = False
                for p, p0 in zip(c["C"], C0):
                    assert np.array_equal(bits(p)[pad], bits(p0)[pad])


def check_cgemm_identities(lib):
    z = ((0.0, 0.0), (0.0, 0.0))
    one = ((1.0, 0.0), (0.0, 0.0))
    # 1. transposed and conjugate-transposed copies give the same bits
    c = W.cgemm_case(3100, "N", "N", 5, 4, 6, dist="wide", padded=False)
    ref = tuple(p.copy() for p in c["C"])
    assert oracle.cgemm("N", "N", 5, 4, 6, c["alpha"], c["A"], 5, c["B"], 6, c["beta"], ref, 5,
                        lib=lib) == 0

    def copy_as(P, rows, cols, t):
        M = [p[: rows * cols].reshape(rows, cols, order="F") for p in P]
        if t == "N":
            return tuple(colmajor(m) for m in M)
        out = [colmajor(m.T) for m in M]
        if t == "C":
            out[2], out[3] = -out[2], -out[3]
        return tuple(out)
    for ta, tb in W.COPS:
        A = copy_as(c["A"], 5, 6, ta)
        B = copy_as(c["B"], 6, 4, tb)
        Cw = tuple(p.copy() for p in c["C"])
        assert oracle.cgemm(ta, tb, 5, 4, 6, c["alpha"], A, 5 if ta == "N" else 6, B,
                            6 if tb == "N" else 4, c["beta"], Cw, 5, lib=lib) == 0
        for p, q in zip(Cw, ref):
            assert np.array_equal(bits(p), bits(q)), (ta, tb)
    # 2. real data: the real parts equal the real oracle's result, imaginary parts 0
    g = W.gemm_case(3101, "T", "N", 6, 5, 7, dist="wide")
    zA, zB, zC = (np.zeros_like(g["A"][0]),) * 2, (np.zeros_like(g["B"][0]),) * 2, \
        (np.zeros_like(g["C"][0]),) * 2
    Cc = (g["C"][0].copy(), g["C"][1].copy()) + tuple(x.copy() for x in zC)
    Rr = (g["C"][0].copy(), g["C"][1].copy())
    for t in ("T", "C"):
        Cw = tuple(p.copy() for p in Cc)
        assert oracle.cgemm(t, "N", 6, 5, 7, (g["alpha"], (0.0, 0.0)), g["A"] + zA, g["lda"],
                            g["B"] + zB, g["ldb"], (g["beta"], (0.0, 0.0)), Cw, g["ldc"],
                            lib=lib) == 0
        if t == "T":
            assert oracle.rgemm("T", "N", 6, 5, 7, g["alpha"], g["A"], g["lda"], g["B"],
                                g["ldb"], g["beta"], Rr, g["ldc"], lib=lib) == 0
        i, j = np.meshgrid(np.arange(6), np.arange(5), indexing="ij")
        idx = (i + j * g["ldc"]).ravel()
        assert np.array_equal(Cw[0][idx], Rr[0][idx]) and np.array_equal(Cw[1][idx], Rr[1][idx])
        assert not Cw[2][idx].any() and not Cw[3][idx].any()
    # 3. alpha = 0, beta = 1: quick return, C bit-identical (NaN sentinel kept)
    c = W.cgemm_case(3102, "N", "C", 4, 4, 4, c_nan=True)
    Cw = tuple(p.copy() for p in c["C"])
    assert oracle.cgemm("N", "C", 4, 4, 4, z, c["A"], c["lda"], c["B"], c["ldb"], one, Cw,
                        c["ldc"], lib=lib) == 0
    for p, q in zip(Cw, c["C"]):
        assert np.array_equal(bits(p), bits(q))
    # 4. beta = 0: C (all NaN) is not read; alpha = 0 as well gives exact zeros
    for alpha in (c["alpha"], z):
        Cw = tuple(p.copy() for p in c["C"])
        assert oracle.cgemm("N", "C", 4, 4, 4, alpha, c["A"], c["lda"], c["B"], c["ldb"], z, Cw,
                            c["ldc"], lib=lib) == 0
        i, j = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
        idx = (i + j * c["ldc"]).ravel()
        for p in Cw:
            assert np.all(np.isfinite(p[idx]))
            if alpha is z:
                assert not p[idx].any()
    # 4b. alpha = 0 with a complex beta of real part 1: C <- beta C (not a quick
    # return), checked against the exact product
    bq = ((1.0, 0.0), (0.5, 0.0))
    c = W.cgemm_case(3104, "N", "N", 3, 3, 3)
    Cw = tuple(p.copy() for p in c["C"])
    assert oracle.cgemm("N", "N", 3, 3, 3, z, c["A"], c["lda"], c["B"], c["ldb"], bq, Cw,
                        c["ldc"], lib=lib) == 0
    for j in range(3):
        for i in range(3):
            o = i + j * c["ldc"]
            re, im = F(c["C"][0][o], c["C"][1][o]), F(c["C"][2][o], c["C"][3][o])
            ex = (re - Fraction(1, 2) * im, im + Fraction(1, 2) * re)
            got = (F(Cw[0][o], Cw[1][o]), F(Cw[2][o], Cw[3][o]))
            for q in range(2):
                assert abs(got[q] - ex[q]) <= 20 * U2 * (abs(re) + abs(im)), (i, j, q)
    # 5. identity: A = I, alpha = 1, beta = 0 gives op(B) bit-exactly
    n = 4
    b = W.cgemm_case(3103, "N", "C", n, n, n, padded=False)
    I = (np.eye(n).ravel(order="F"), np.zeros(n * n), np.zeros(n * n), np.zeros(n * n))
    Cw = tuple(np.zeros(n * n) for _ in range(4))
    assert oracle.cgemm("N", "C", n, n, n, one, I, n, b["B"], n, z, Cw, n, lib=lib) == 0
    Bh = [p.reshape(n, n, order="F").T.ravel(order="F") for p in b["B"]]
    assert np.array_equal(Cw[0], Bh[0]) and np.array_equal(Cw[1], Bh[1])
    assert np.array_equal(Cw[2], -Bh[2]) and np.array_equal(Cw[3], -Bh[3])


def check_cgemm_info_codes(lib):
    pos = read_arg_positions()
    z = ((0.0, 0.0), (0.0, 0.0))
    C = tuple(np.zeros(16) for _ in range(4))
    N = (None,) * 4

    def info(ta="N", tb="N", m=2, n=2, k=2, lda=None, ldb=None, ldc=None):
        lda = lda if lda is not None else max(1, m if ta == "N" else k)
        ldb = ldb if ldb is not None else max(1, k if tb == "N" else n)
        ldc = ldc if ldc is not None else max(1, m)
        return oracle.cgemm(ta, tb, m, n, k, ((1.0, 0.0), (0.0, 0.0)), N, lda, N, ldb, z, C, ldc,
                            lib=lib)
    assert info(ta="X") == pos[("gemm", "transa")]
    assert info(tb="Q") == pos[("gemm", "transb")]
    assert info(m=-1) == pos[("gemm", "m")]
    assert info(n=-1) == pos[("gemm", "n")]
    assert info(k=-1) == pos[("gemm", "k")]
    assert info(ta="C", m=3, k=2, lda=1) == pos[("gemm", "lda")]
    assert info(tb="C", n=3, k=2, ldb=2) == pos[("gemm", "ldb")]
    assert info(m=3, ldc=2) == pos[("gemm", "ldc")]


# ---- dd division, square root and the Cholesky factorisation Rpotrf ------------------

def check_div_sqrt(lib, count=300):
    rng = np.random.default_rng(11)
    for dist in ("uniform", "wide"):
        xh, xl = W.dd_values(rng, count, dist)
        yh, yl = W.dd_values(rng, count, dist)
        for t in range(count):
            if yh[t] == 0.0:
                continue
            x, y = F(xh[t], xl[t]), F(yh[t], yl[t])
            z = F(*oracle.dd_div((xh[t], xl[t]), (yh[t], yl[t]), lib=lib))
            q = x / y
            assert abs(z - q) <= 16 * U2 * abs(q), ("div", dist, t)
            # square root of |x|: (z - e)^2 <= |x| <= (z + e)^2 with e = 3.2 u^2 z
            a = abs(x)
            if a == 0:
                continue
            ah, al = (xh[t], xl[t]) if xh[t] > 0 else (-xh[t], -xl[t])
            s = F(*oracle.dd_sqrt((ah, al), lib=lib))
            e = Fraction(32, 10) * U2 * s
            assert (s - e) ** 2 <= a <= (s + e) ** 2, ("sqrt", dist, t)
    # exact cases
    for (x, y, q) in ((6.0, 3.0, 2.0), (1.0, 4.0, 0.25), (7.0, 7.0, 1.0), (-9.0, 3.0, -3.0)):
        assert oracle.dd_div((x, 0.0), (y, 0.0), lib=lib) == (q, 0.0)
    for (x, r) in ((4.0, 2.0), (2.25, 1.5), (1.0, 1.0)):
        assert oracle.dd_sqrt((x, 0.0), lib=lib) == (r, 0.0)
    # (1 + 2^-40)^2 = 1 + 2^-39 + 2^-80: needs the low part to come out exact
    assert oracle.dd_sqrt((1.0 + 2.0 ** -39, 2.0 ** -80), lib=lib) == (1.0 + 2.0 ** -40, 0.0)


def _tri_full(M, n, ld, uplo):
    """Column-major (hi, lo) planes of ld x n holding the uplo triangle of the
    symmetric n x n array M (a list of (hi, lo) rows); the other triangle and
    the padding rows hold the NaN sentinel."""
    hi = np.full(ld * n, W.SENTINEL_HI)
    lo = np.full(ld * n, W.SENTINEL_LO)
    for i in range(n):
        for j in range(n):
            if (uplo == "L" and i >= j) or (uplo == "U" and i <= j):
                hi[i + j * ld], lo[i + j * ld] = M[i][j]
    return hi, lo


def check_potrf_exact_integer(lib):
    """A = L L^T with small integer L (positive diagonal): every quantity is an
    integer, so both triangles come out exactly L (lo parts 0)."""
    rng = np.random.default_rng(12)
    for n in (1, 2, 5, 9, 12):
        L = np.tril(rng.integers(-3, 4, (n, n))).astype(np.int64)
        np.fill_diagonal(L, rng.integers(1, 5, n))
        A = L @ L.T
        M = [[(float(A[i, j]), 0.0) for j in range(n)] for i in range(n)]
        for uplo in "LU":
            ld = n + 2
            hi, lo = _tri_full(M, n, ld, uplo)
            h0, l0 = hi.copy(), lo.copy()
            assert oracle.rpotrf(uplo, n, (hi, lo), ld, lib=lib) == 0
            for i in range(n):
                for j in range(n):
                    o = i + j * ld
                    inside = (i >= j) if uplo == "L" else (i <= j)
                    if inside:
                        want = L[i, j] if uplo == "L" else L[j, i]
                        assert hi[o] == want and lo[o] == 0.0, (n, uplo, i, j)
                    else:
                        assert bits(hi[o:o + 1])[0] == bits(h0[o:o + 1])[0]
                        assert bits(lo[o:o + 1])[0] == bits(l0[o:o + 1])[0]
            pad = np.ones(ld * n, bool)
            for j in range(n):
                pad[j * ld: j * ld + n] = False
            assert np.array_equal(bits(hi)[pad], bits(h0)[pad])


def spd_matrix(rng, n, dist="uniform"):
    """Symmetric positive definite dd matrix B B^T / n + I with dd-random B,
    rounded to dd; returns an n x n list of (hi, lo)."""
    bh, bl = W.dd_values(rng, n * n, dist if dist != "wide" else "uniform")
    B = [[F(bh[i * n + j], bl[i * n + j]) for j in range(n)] for i in range(n)]
    M = []
    for i in range(n):
        row = []
        for j in range(n):
            v = sum((B[i][l] * B[j][l] for l in range(n)), Fraction(0)) / n
            if i == j:
                v += 1
            h = float(v)
            row.append((h, float(v - Fraction(h))))
        M.append(row)
    for i in range(n):                 # exactly symmetric
        for j in range(i):
            M[j][i] = M[i][j]
    return M


def potrf_bound(n):
    """Entrywise backward-error bound of the dd Cholesky in units of
    (|L| |L|^T)_ij: each of the <= n subtracted products and sums costs at most
    7 u^2, the square root 25/8 u^2 and the quotient 16 u^2."""
    return (7 * n + 40) * U2


def check_potrf_residual(lib, sizes=(1, 3, 6, 8)):
    rng = np.random.default_rng(13)
    for n in sizes:
        M = spd_matrix(rng, n)
        for uplo in "LU":
            ld = n + 1
            hi, lo = _tri_full(M, n, ld, uplo)
            assert oracle.rpotrf(uplo, n, (hi, lo), ld, lib=lib) == 0

            def Lv(i, l):
                if i < l:
                    return Fraction(0)
                o = (i + l * ld) if uplo == "L" else (l + i * ld)
                return F(hi[o], lo[o])
            bnd = potrf_bound(n)
            for i in range(n):
                for j in range(i + 1):
                    s = sum((Lv(i, l) * Lv(j, l) for l in range(n)), Fraction(0))
                    mag = sum((abs(Lv(i, l) * Lv(j, l)) for l in range(n)), Fraction(0))
                    a = F(*M[i][j])
                    assert abs(s - a) <= bnd * mag, (n, uplo, i, j, float(abs(s - a) / mag))
                    if i == j:
                        assert Lv(i, i) > 0


def check_potrf_transpose_and_info(lib):
    rng = np.random.default_rng(14)
    n, ld = 7, 9
    M = spd_matrix(rng, n)
    hl, ll = _tri_full(M, n, ld, "L")
    hu, lu = _tri_full(M, n, ld, "U")
    assert oracle.rpotrf("L", n, (hl, ll), ld, lib=lib) == 0
    assert oracle.rpotrf("u", n, (hu, lu), ld, lib=lib) == 0
    for i in range(n):
        for j in range(i + 1):
            a, b = i + j * ld, j + i * ld
            assert bits(hl[a:a + 1])[0] == bits(hu[b:b + 1])[0]
            assert bits(ll[a:a + 1])[0] == bits(lu[b:b + 1])[0]
    # not positive definite at order k: info = k, earlier columns factored
    for k in (1, 3, 7):
        Mk = [[(1.0 if i == j else 0.0, 0.0) for j in range(n)] for i in range(n)]
        Mk[k - 1][k - 1] = (-1.0, 0.0)
        h, l = _tri_full(Mk, n, ld, "L")
        assert oracle.rpotrf("L", n, (h, l), ld, lib=lib) == k
        assert h[(k - 1) * (ld + 1)] == -1.0
    # a zero pivot after elimination: [[1, 1], [1, 1]] -> info 2
    h, l = _tri_full([[(1.0, 0.0), (1.0, 0.0)], [(1.0, 0.0), (1.0, 0.0)]], 2, 2, "U")
    assert oracle.rpotrf("U", 2, (h, l), 2, lib=lib) == 2
    # NaN on the diagonal
    Mk = [[(1.0 if i == j else 0.0, 0.0) for j in range(3)] for i in range(3)]
    Mk[1][1] = (float("nan"), 0.0)
    h, l = _tri_full(Mk, 3, 3, "L")
    assert oracle.rpotrf("L", 3, (h, l), 3, lib=lib) == 2
    # LAPACK argument errors (negative positions), nothing written
    h = np.full(4, 5.0)
    l = np.zeros(4)
    assert oracle.rpotrf("X", 2, (h, l), 2, lib=lib) == -1
    assert oracle.rpotrf("L", -1, (h, l), 2, lib=lib) == -2
    assert oracle.rpotrf("L", 2, (h, l), 1, lib=lib) == -4
    assert oracle.rpotrf("L", 0, (h, l), 1, lib=lib) == 0
    assert np.all(h == 5.0)


# ---- quad-double Rgemm -----------------------------------------------------------------

def qd_of(v):
    """Greedy nearest rounding of an exact rational to a qd: x0 = RN(v),
    x1 = RN(v - x0), ... (Python's float() of a Fraction rounds to nearest,
    ties to even)."""
    out = []
    for _ in range(4):
        x = float(v)
        out.append(x)
        v = v - Fraction(x)
    return tuple(out)


def QF(*parts):
    return sum((Fraction(float(p)) for p in parts), Fraction(0))


def check_qd_round(lib, count=200):
    rng = np.random.default_rng(21)
    for t in range(count):
        n = int(rng.integers(1, 12))
        e = rng.integers(-200, 60, n)
        terms = np.ldexp(rng.uniform(-1.0, 1.0, n), e)
        if t % 5 == 0:                       # heavy cancellation
            terms = np.concatenate([terms, -terms[:1] * (1 + 2.0 ** -50)])
        want = qd_of(sum((Fraction(float(x)) for x in terms), Fraction(0)))
        got = oracle.qd_round_sum(terms, lib=lib)
        assert got == want, (t, got, want)
    assert oracle.qd_round_sum([0.1, 0.2], lib=lib) == (0.30000000000000004, -2.7755575615628914e-17,
                                                       0.0, 0.0)
    # ties to even on the last part: 1 + 2^-53 rounds to 1, remainder 2^-53 exactly
    assert oracle.qd_round_sum([1.0, 2.0 ** -53], lib=lib) == (1.0, 2.0 ** -53, 0.0, 0.0)
    assert oracle.qd_round_sum([], lib=lib) == (0.0, 0.0, 0.0, 0.0)


def check_qgemm_exact(lib, seeds=range(2), dist="uniform",
                      sizes=((1, 1, 1), (2, 3, 4), (4, 3, 2), (3, 2, 5))):
    """Every entry of the oracle's qd Rgemm equals the greedy nearest qd of the
    exact result (Fraction arithmetic), bit for bit, in all four op forms;
    padding rows are untouched."""
    for seed in seeds:
        for (m, n, k) in sizes:
            for ta in "NT":
                for tb in "NT":
                    c = W.qgemm_case(6000 + seed, ta, tb, m, n, k, dist=dist)
                    C0 = tuple(p.copy() for p in c["C"])
                    assert oracle.qgemm(ta, tb, m, n, k, c["alpha"], c["A"], c["lda"], c["B"],
                                        c["ldb"], c["beta"], c["C"], c["ldc"], lib=lib) == 0
                    al, be = QF(*c["alpha"]), QF(*c["beta"])

                    def op(P, ld, t, r, q):
                        idx = (q + r * ld) if t == "T" else (r + q * ld)
                        return QF(*(p[idx] for p in P))
                    for i in range(m):
                        for j in range(n):
                            o = i + j * c["ldc"]
                            dot = sum((op(c["A"], c["lda"], ta, i, l) * op(c["B"], c["ldb"], tb, l, j)
                                       for l in range(k)), Fraction(0))
                            want = qd_of(al * dot + be * QF(*(p[o] for p in C0)))
                            got = tuple(float(p[o]) for p in c["C"])
                            assert got == want, (seed, m, n, k, ta, tb, i, j)
                    ldc = c["ldc"]
                    pad = np.ones(ldc * n, bool)
                    for j in range(n):
                        pad[j * ldc: j * ldc + m] = False
                    for p, p0 in zip(c["C"], C0):
                        assert np.array_equal(bits(p)[pad], bits(p0)[pad])


def check_qgemm_semantics(lib):
    """The worked Rgemm example in qd (integer data: exact), quick returns,
    beta = 0 with a NaN C, alpha = 0, and the BLAS argument positions."""
    alpha, beta, v = read_worked_example()
    z = np.zeros(9)
    for ta in "NT":
        for tb in "NT":
            A = colmajor(v["A"] if ta == "N" else v["A"].T)
            B = colmajor(v["B"] if tb == "N" else v["B"].T)
            C = (colmajor(v["C"]), z.copy(), z.copy(), z.copy())
            assert oracle.qgemm(ta, tb, 3, 3, 3, (alpha, 0, 0, 0), (A, z, z, z), 3,
                                (B, z, z, z), 3, (beta, 0, 0, 0), C, 3, lib=lib) == 0
            assert np.array_equal(C[0], colmajor(v["ANSWER"]))
            assert not C[1].any() and not C[2].any() and not C[3].any()
    c = W.qgemm_case(6100, "N", "T", 5, 4, 3, c_nan=True)
    one, zero = (1.0, 0.0, 0.0, 0.0), (0.0,) * 4
    # alpha = 0, beta = 1: quick return, C bit-identical
    Cw = tuple(p.copy() for p in c["C"])
    assert oracle.qgemm("N", "T", 5, 4, 3, zero, c["A"], c["lda"], c["B"], c["ldb"], one, Cw,
                        c["ldc"], lib=lib) == 0
    for p, q in zip(Cw, c["C"]):
        assert np.array_equal(bits(p), bits(q))
    # beta = 0: NaN C not read; with alpha = 0 as well the result is exactly 0
    for al in (c["alpha"], zero):
        Cw = tuple(p.copy() for p in c["C"])
        assert oracle.qgemm("N", "T", 5, 4, 3, al, c["A"], c["lda"], c["B"], c["ldb"], zero, Cw,
                            c["ldc"], lib=lib) == 0
        i, j = np.meshgrid(np.arange(5), np.arange(4), indexing="ij")
        idx = (i + j * c["ldc"]).ravel()
        for p in Cw:
            assert np.all(np.isfinite(p[idx]))
            if al is zero:
                assert not p[idx].any()
    pos = read_arg_positions()
    N4 = (None,) * 4
    C4 = tuple(np.zeros(9) for _ in range(4))

    def info(ta="N", tb="N", m=2, n=2, k=2, lda=None, ldb=None, ldc=None):
        lda = lda if lda is not None else max(1, m if ta == "N" else k)
        ldb = ldb if ldb is not None else max(1, k if tb == "N" else n)
        ldc = ldc if ldc is not None else max(1, m)
        return oracle.qgemm(ta, tb, m, n, k, one, N4, lda, N4, ldb, zero, C4, ldc, lib=lib)
    assert info(ta="X") == pos[("gemm", "transa")]
    assert info(tb="q") == pos[("gemm", "transb")]
    assert info(m=-1) == pos[("gemm", "m")]
    assert info(n=-1) == pos[("gemm", "n")]
    assert info(k=-1) == pos[("gemm", "k")]
    assert info(m=3, lda=2) == pos[("gemm", "lda")]
    assert info(k=3, ldb=2) == pos[("gemm", "ldb")]
    assert info(m=3, lda=3, ldc=2) == pos[("gemm", "ldc")]

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

def check_ozaki_split_exact(lib, dist="wide", nslices=18):
    """Digits reconstruct the scaled value exactly up to the last remainder,
    stay within their bounds, and the scale puts every row inside (-1, 1)."""
    for (rows, k, trans) in [(5, 7, False), (4, 9, True), (1, 1, False)]:
        rng = W.streams(4000 + rows)[0]
        ld = rows + 2 if not trans else k + 1
        nr, nc = (rows, k) if not trans else (k, rows)
        X = W.dd_matrix(rng, nr, nc, ld, dist=dist)
        sr, sl = (1, ld) if not trans else (ld, 1)
        for (wf, w) in (oracle.INT8_DIGITS, oracle.fp64_digit_width(k, nslices)):
            exps, digs = oracle.ozaki_split(rows, k, X, sr, sl, nslices, wf, w, lib=lib)
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
                        lim = 2 ** wf if t == 0 else 2 ** (w - 1)
                        assert abs(q) <= lim, (t, q, lim)
                        W_t = wf + w * t
                        recon += Fraction(q, 2 ** W_t)
                        # remainder after digit t lies within half a unit of it
                        assert abs(x - recon) <= Fraction(1, 2 ** (W_t + 1)) * Fraction(
                            1000001, 1000000), (t, float(x - recon))


def check_ozaki_gemm_exact(lib):
    """Split-form result vs exact rational arithmetic on the same digits: the
    recombination of the kept anti-diagonals must match the exact sum of the
    kept digit products to within the dd rounding of the final steps."""
    m, n, k, s = 4, 3, 5, 6
    for ta in "NT":
        for tb in "NT":
            c = W.gemm_case(5000, ta, tb, m, n, k, dist="wide")
            for (wf, w) in (oracle.INT8_DIGITS, oracle.fp64_digit_width(k, s)):
                C = (c["C"][0].copy(), c["C"][1].copy())
                C0 = (c["C"][0].copy(), c["C"][1].copy())
                assert oracle.ozaki_rgemm(ta, tb, m, n, k, c["alpha"], c["A"], c["lda"], c["B"],
                                          c["ldb"], c["beta"], C, c["ldc"], s, wf, w,
                                          lib=lib) == 0
                ea, qa = oracle.ozaki_split(m, k, c["A"], c["lda"] if ta == "T" else 1,
                                            1 if ta == "T" else c["lda"], s, wf, w, lib=lib)
                eb, qb = oracle.ozaki_split(n, k, c["B"], 1 if tb == "T" else c["ldb"],
                                            c["ldb"] if tb == "T" else 1, s, wf, w, lib=lib)
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

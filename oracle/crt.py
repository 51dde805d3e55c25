"""CPU oracle for the modular (Chinese-remainder) split form of dd Rgemm --
TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; it shares no code with the GPU library.  Exact integers
are Python ints; numpy serves for the float64 steps and for the per-modulus
integer products.  Small sizes only (Python-integer arrays).

The manual has no split method.  This form follows the integer modular
emulation of a floating-point matrix product by Ozaki, Uchino and Imamura
(Ozaki scheme II, 2025), applied to dd operands:

1. Scale.  sigma_r: the frexp exponent of the largest |hi| of row r of the
   row operand (a row of op(A), or a column of op(B)); |x_rl| < 2^sigma_r.
   An all-zero row gets 0.
2. Integers.  With P bits (`exponent`), z = x 2^(P - sigma) (exact, two
   binary64 parts zh, zl); t1 = rint(zh), t2 = rint((zh - t1) + zl) in
   binary64 (ties to even); the integer is X' = t1 + t2, within 1/2 + 2^-52 of
   z, so |X'| <= 2^P.
3. Residues.  For each modulus m of the list (`moduli`: the largest first,
   each pairwise coprime to those before it), the balanced residue of X'
   modulo m: the representative in [-(m-1)/2, (m-1)/2] for odd m, in
   [-128, 127] for m = 256.  All fit int8.
4. Products.  For each modulus, R_A R_B^T over the k terms, exact in
   integers (|.| <= k 2^14).
5. Reconstruction.  The unique X in [-M/2, M/2) (M the product of the
   moduli) congruent to every product modulo its modulus.  P is chosen so
   that 4 k 2^(2P) <= M; then X equals the exact integer product
   sum_l A'_il B'_jl.
6. Result.  C = alpha (X 2^(sigma_i + tau_j - 2P)) + beta C, evaluated exactly
   and rounded to the nearest dd (hi nearest binary64, lo nearest binary64 of
   the rest).

Complex operands (crt_cgemm): the real and imaginary parts of a row share
one exponent (that of the largest |hi| over both parts), each part becomes
its grid integers (a conjugated operand negates the imaginary integers), and
with T1 = Ar' Br'^T, T2 = Ai' Bi'^T, T3 = (Ar' + Ai')(Br' + Bi')^T (three
exact integer products) the product is Re X = T1 - T2, Im X = T3 - T1 - T2,
both exact; |Re X|, |Im X| <= 2 k 2^(2P), so P follows 8 k 2^(2P) <= M.
Each part is reconstructed from its residues (T1 - T2 and T3 - T1 - T2
modulo every modulus); then C = alpha X 2^(sigma_i + tau_j - 2P) + beta C in
exact complex arithmetic, each part rounded to the nearest dd.
"""
from fractions import Fraction
from math import gcd

import numpy as np

MAX_MODULI = 32     # the most moduli the form uses
MAX_BITS = 104      # the widest integer grid: t2 and the chunks of X' stay exact


def moduli(count):
    """The first `count` moduli: from 256 downward, every integer that is
    coprime to all moduli taken before it (step 3)."""
    if count < 1 or count > MAX_MODULI:
        raise ValueError("count out of range")
    out = []
    m = 256
    while len(out) < count:
        if all(gcd(m, q) == 1 for q in out):
            out.append(m)
        m -= 1
    return out


def modulus_product(count):
    M = 1
    for m in moduli(count):
        M *= m
    return M


def exponent(k, count, margin_bits=2):
    """P (step 5): the largest P <= MAX_BITS with 2^margin_bits k 2^(2P) <= M
    (margin 2 for real products, 3 for complex ones), or None when there is
    none >= 1."""
    M = modulus_product(count)
    lk = max(0, (max(k, 1) - 1).bit_length())       # ceil(log2 k)
    p = ((M.bit_length() - 1) - margin_bits - lk) // 2
    p = min(p, MAX_BITS)
    return p if p >= 1 else None


def scale_exponents(hi_rows):
    """Step 1 for a (rows x k) float64 array of leading parts."""
    mx = np.max(np.abs(hi_rows), axis=1) if hi_rows.shape[1] else np.zeros(hi_rows.shape[0])
    _, e = np.frexp(mx)
    return np.where(mx == 0.0, 0, e).astype(np.int64)


_to_int = np.frompyfunc(int, 1, 1)     # elementwise exact float -> Python int


def integers(hi_rows, lo_rows, exps, p):
    """Step 2: the integers X' (Python ints, object array rows x k)."""
    sh = (p - exps).astype(np.int64)[:, None]
    zh = np.ldexp(hi_rows, sh)
    zl = np.ldexp(lo_rows, sh)
    t1 = np.rint(zh)
    t2 = np.rint((zh - t1) + zl)
    return _to_int(t1) + _to_int(t2)


def balanced(x, m):
    """Step 3's representative modulo m of x (a Python int, or an object
    array of them, elementwise)."""
    r = x % m
    top = (m - 1) // 2 if m % 2 else m // 2 - 1      # largest representative
    return np.where(r > top, r - m, r) if isinstance(r, np.ndarray) else (r - m if r > top else r)


def residues(ints, count):
    """Step 3: int64 array (count, rows, k) of balanced residues."""
    ms = moduli(count)
    out = np.zeros((count,) + ints.shape, dtype=np.int64)
    for t, m in enumerate(ms):
        out[t] = balanced(ints, m).astype(np.int64)
    return out


def reconstruct(prods, count):
    """Step 5: prods[t] congruent to X modulo modulus t -- Python ints, or
    integer arrays of one shape (then elementwise, Python ints out)."""
    ms = moduli(count)
    M = modulus_product(count)
    x = 0
    for r, m in zip(prods, ms):
        Mt = M // m
        r = np.asarray(r).astype(object) if isinstance(r, np.ndarray) else int(r)
        x = x + r * (Mt * pow(Mt, -1, m))
    x = x % M
    half = (M + 1) // 2
    return np.where(x >= half, x - M, x) if isinstance(x, np.ndarray) else (x - M if x >= half else x)


def row_operand(trans, rows, k, X, ld):
    """Row operand (rows x k) of a column-major dd matrix: trans 'N' takes
    element (r, l) from X[r + l ld], 'T' from X[l + r ld]."""
    hi, lo = X
    r = np.arange(rows)[:, None]
    l = np.arange(k)[None, :]
    idx = (r + l * ld) if trans.upper() == "N" else (l + r * ld)
    return hi[idx], lo[idx]


def _nearest_dd(v):
    h = float(v)
    return h, float(v - Fraction(h))


def integer_product(transa, transb, m, n, k, A, lda, B, ldb, count):
    """Steps 1-5: exponents (sigma, tau), P and the exact integer product X
    (object array m x n) obtained from the residue products."""
    p = exponent(k, count)
    if p is None:
        raise ValueError("too few moduli for k")
    ah, al = row_operand(transa, m, k, A, lda)
    bt = "T" if transb.upper() == "N" else "N"   # columns of op(B) as rows
    bh, bl = row_operand(bt, n, k, B, ldb)
    ea, eb = scale_exponents(ah), scale_exponents(bh)
    ra = residues(integers(ah, al, ea, p), count)
    rb = residues(integers(bh, bl, eb, p), count)
    prods = [ra[t] @ rb[t].T for t in range(count)]  # exact in int64
    return ea, eb, p, reconstruct(prods, count)


def crt_rgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, count):
    """Step 6 on top of integer_product: C updated in place (column-major
    planes C = (hi, lo), leading dimension ldc); returns C."""
    ch, cl = C
    if m == 0 or n == 0:
        return C
    a = Fraction(alpha[0]) + Fraction(alpha[1])
    b = Fraction(beta[0]) + Fraction(beta[1])
    if k == 0 or a == 0:
        ea = eb = None
        p = 0
        X = np.zeros((m, n), dtype=object)
    else:
        ea, eb, p, X = integer_product(transa, transb, m, n, k, A, lda, B, ldb, count)
    for j in range(n):
        for i in range(m):
            v = Fraction(0)
            if X[i, j]:
                v = a * X[i, j] * Fraction(2) ** int(ea[i] + eb[j] - 2 * p)
            if b != 0:
                v += b * (Fraction(ch[i + j * ldc]) + Fraction(cl[i + j * ldc]))
            ch[i + j * ldc], cl[i + j * ldc] = _nearest_dd(v)
    return C


def complex_row_operand(trans, rows, k, X, ld):
    """Row operand of a complex matrix X = (re.hi, re.lo, im.hi, im.lo) as
    (re hi, re lo, im hi, im lo) arrays rows x k; trans 'C' conjugates."""
    rh, rl = row_operand("N" if trans.upper() == "N" else "T", rows, k, X[:2], ld)
    ih, il = row_operand("N" if trans.upper() == "N" else "T", rows, k, X[2:], ld)
    if trans.upper() == "C":
        ih, il = -ih, -il
    return rh, rl, ih, il


def complex_scale_exponents(rh, ih):
    """One exponent per row over both parts: that of the largest |hi|."""
    return scale_exponents(np.concatenate([rh, ih], axis=1))


def complex_integer_product(transa, transb, m, n, k, A, lda, B, ldb, count):
    """Exponents, P and the exact integer parts (Re X, Im X) of the complex
    product, from the residues of the three products T1, T2, T3."""
    p = exponent(k, count, margin_bits=3)
    if p is None:
        raise ValueError("too few moduli for k")
    ms = moduli(count)
    arh, arl, aih, ail = complex_row_operand(transa, m, k, A, lda)
    # columns of op(B) as rows: op(B) = B ('N'), B^T ('T'), conj(B)^T ('C')
    bt = {"N": "T", "T": "N", "C": "C"}[transb.upper()]
    if bt == "C":
        brh, brl, bih, bil = complex_row_operand("N", n, k, B, ldb)
        bih, bil = -bih, -bil
    else:
        brh, brl, bih, bil = complex_row_operand(bt, n, k, B, ldb)
    ea, eb = complex_scale_exponents(arh, aih), complex_scale_exponents(brh, bih)
    Ar, Ai = integers(arh, arl, ea, p), integers(aih, ail, ea, p)
    Br, Bi = integers(brh, brl, eb, p), integers(bih, bil, eb, p)
    ra, ia, sa = residues(Ar, count), residues(Ai, count), residues(Ar + Ai, count)
    rb, ib, sb = residues(Br, count), residues(Bi, count), residues(Br + Bi, count)
    re, im = [], []
    for t in range(count):
        t1, t2, t3 = ra[t] @ rb[t].T, ia[t] @ ib[t].T, sa[t] @ sb[t].T
        re.append(t1 - t2)
        im.append(t3 - t1 - t2)
    return ea, eb, p, reconstruct(re, count), reconstruct(im, count)


def crt_cgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, count):
    """Complex form of crt_rgemm: A, B, C are (re.hi, re.lo, im.hi, im.lo)
    column-major planes, alpha and beta ((re.hi, re.lo), (im.hi, im.lo));
    C updated in place and returned."""
    crh, crl, cih, cil = C
    if m == 0 or n == 0:
        return C
    fr = lambda x: Fraction(x[0]) + Fraction(x[1])
    ar, ai = fr(alpha[0]), fr(alpha[1])
    br, bi = fr(beta[0]), fr(beta[1])
    if k == 0 or (ar == 0 and ai == 0):
        ea = eb = None
        p = 0
        XR = XI = np.zeros((m, n), dtype=object)
    else:
        ea, eb, p, XR, XI = complex_integer_product(transa, transb, m, n, k, A, lda, B, ldb,
                                                    count)
    for j in range(n):
        for i in range(m):
            vr = vi = Fraction(0)
            if XR[i, j] or XI[i, j]:
                sc = Fraction(2) ** int(ea[i] + eb[j] - 2 * p)
                pr, pi = XR[i, j] * sc, XI[i, j] * sc
                vr, vi = ar * pr - ai * pi, ar * pi + ai * pr
            if br != 0 or bi != 0:
                q = i + j * ldc
                cr = Fraction(crh[q]) + Fraction(crl[q])
                ci = Fraction(cih[q]) + Fraction(cil[q])
                vr += br * cr - bi * ci
                vi += br * ci + bi * cr
            q = i + j * ldc
            crh[q], crl[q] = _nearest_dd(vr)
            cih[q], cil[q] = _nearest_dd(vi)
    return C


# ---- quad-double operands ------------------------------------------------------------
#
# A qd entry x = x0 + x1 + x2 + x3 (four binary64 parts) of row r becomes
# the integer X' = sum_p rint(x_p 2^(QD_GRID_BITS - sigma_r)) (sigma_r from
# the row's largest |x0|), |X' - z| <= 2 for the exact scaled value z.  Each
# part's integer t_p is cut into 26-bit chunks from the top (j = 7 .. 1:
# c_j = rint(t 2^(-26 j)), t -= c_j 2^(26 j), exact; c_0 = t), C_j = sum_p c_pj,
# and X' = X1 2^104 + X0 with X0 = sum_{j<4} C_j 2^(26 j), X1 = sum_{j>=4}
# C_j 2^(26 (j - 4)); |X0|, |X1| < 2^105.01.  The product of two such rows is
# A 2^208 + (C - A - B) 2^104 + B with A = X1 Y1, B = X0 Y0 and
# C = (X1 + X0)(Y1 + Y0) (three exact integer products, each below 2^212 k
# in magnitude), every one rebuilt from its residues: the moduli count must
# give M >= 2^(215 + ceil(log2 k)).  The result is rounded to the nearest qd
# greedily (x0 = RN(V), x1 = RN(V - x0), ...).

QD_GRID_BITS = 208
QD_CHUNK_BITS = 26
QD_SPLIT_BITS = 104


def qd_count_ok(k, count):
    """Whether `count` moduli recover the three qd sub-products for k terms."""
    if count < 1 or count > MAX_MODULI:
        return False
    lk = max(0, (max(k, 1) - 1).bit_length())
    return modulus_product(count).bit_length() - 1 >= 215 + lk


def qd_scale_exponents(x0_rows):
    return scale_exponents(x0_rows)


def qd_chunks(parts, exps):
    """The chunk sums C_j (int64 array (8, rows, k)) of the grid integers of a
    qd row operand given as four (rows x k) part arrays."""
    sh = (QD_GRID_BITS - exps).astype(np.int64)[:, None]
    out = np.zeros((8,) + parts[0].shape, dtype=np.int64)
    for x in parts:
        t = np.rint(np.ldexp(x, sh))
        for j in range(7, 0, -1):
            c = np.rint(np.ldexp(t, -QD_CHUNK_BITS * j))
            t = t - np.ldexp(c, QD_CHUNK_BITS * j)
            out[j] += c.astype(np.int64)
        out[0] += t.astype(np.int64)
    return out


def qd_split(chunks):
    """(X1, X0) as object arrays of Python ints from the chunk sums."""
    obj = chunks.astype(object)
    x0 = sum(obj[j] * (1 << (QD_CHUNK_BITS * j)) for j in range(4))
    x1 = sum(obj[j] * (1 << (QD_CHUNK_BITS * (j - 4))) for j in range(4, 8))
    return x1, x0


def qd_row_operand(trans, rows, k, X, ld):
    """The four parts of a qd row operand (rows x k)."""
    r = np.arange(rows)[:, None]
    l = np.arange(k)[None, :]
    idx = (r + l * ld) if trans.upper() == "N" else (l + r * ld)
    return [p[idx] for p in X]


def qd_integer_product(transa, transb, m, n, k, A, lda, B, ldb, count):
    """Exponents and the exact integer product of the grid integers of op(A)
    and op(B), from the residues of the three sub-products."""
    if not qd_count_ok(k, count):
        raise ValueError("too few moduli for k")
    pa = qd_row_operand(transa, m, k, A, lda)
    pb = qd_row_operand("T" if transb.upper() == "N" else "N", n, k, B, ldb)
    ea, eb = qd_scale_exponents(pa[0]), qd_scale_exponents(pb[0])
    a1, a0 = qd_split(qd_chunks(pa, ea))
    b1, b0 = qd_split(qd_chunks(pb, eb))
    ra = [residues(v, count) for v in (a1, a0, a1 + a0)]
    rb = [residues(v, count) for v in (b1, b0, b1 + b0)]
    prods = [[ra[s][t] @ rb[s][t].T for t in range(count)] for s in range(3)]
    hi, lo, mid = (reconstruct(p, count) for p in prods)
    X = hi * (1 << (2 * QD_SPLIT_BITS)) + (mid - hi - lo) * (1 << QD_SPLIT_BITS) + lo
    return ea, eb, X


def _nearest_qd(v):
    out = []
    for _ in range(4):
        h = float(v)
        out.append(h)
        v = v - Fraction(h)
    return out


def crt_qgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, count):
    """qd Rgemm of the modular form: A, B, C four column-major planes, alpha
    and beta 4-tuples of binary64 parts; C updated in place and returned."""
    if m == 0 or n == 0:
        return C
    a = sum(Fraction(x) for x in alpha)
    b = sum(Fraction(x) for x in beta)
    if k == 0 or a == 0:
        ea = eb = None
        X = np.zeros((m, n), dtype=object)
    else:
        ea, eb, X = qd_integer_product(transa, transb, m, n, k, A, lda, B, ldb, count)
    for j in range(n):
        for i in range(m):
            q = i + j * ldc
            v = Fraction(0)
            if X[i, j]:
                v = a * X[i, j] * Fraction(2) ** int(ea[i] + eb[j] - 2 * QD_GRID_BITS)
            if b != 0:
                v += b * sum(Fraction(float(p[q])) for p in C)
            for p, x in zip(C, _nearest_qd(v)):
                p[q] = x
    return C

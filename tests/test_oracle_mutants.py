"""Plant plausible mistakes in copies of the oracle's C sources and check that
the pin suite catches every one of them (CPU only; the real oracle is never
modified).  This shows the pins are strong enough to trust the oracle."""
import os
import shutil
import tempfile

import pytest

import oracle
import pins
from oracle import build as obuild

SRC = os.path.dirname(os.path.abspath(oracle.__file__))
SOURCES = list(obuild.SOURCES)

# (file, original text, planted mistake, what it models)
MUTANTS = [
    ("dd_ops.h", "double e = (a - (s - bb)) + (b - bb);",
     "double e = (a - (s - bb)) - (b - bb);", "sign error in TwoSum"),
    ("dd_ops.h", "double e = fma(a, b, -p);", "double e = fma(a, b, p);",
     "sign error in TwoProd"),
    ("dd_ops.h", "double e = b - (s - a);", "double e = (s - a) - b;",
     "sign error in FastTwoSum"),
    ("dd_ops.h", "double c2 = fma(x.lo, y.hi, t1);", "double c2 = fma(x.lo, y.lo, t1);",
     "wrong operand in a dd-mul cross term"),
    ("dd_ops.h", "double t1 = fma(x.hi, y.lo, t0);", "double t1 = t0;",
     "dropped dd-mul cross term"),
    ("dd_ops.h", "double w = t.lo + v.lo;", "double w = v.lo;",
     "dropped low-part error in dd add"),
    ("dd_ops.h", "double v = x.lo + s.lo;", "double v = s.lo;",
     "dropped low part in dd + double"),
    ("dd_oracle.c", "int64_t idx = trans ? (c + r * ld) : (r + c * ld);",
     "int64_t idx = trans ? (r + c * ld) : (c + r * ld);", "transposed operand"),
    ("dd_oracle.c", "for (l = 0; l < k; ++l) {", "for (l = 1; l < k; ++l) {",
     "dropped first term"),
    ("dd_oracle.c", "return dd_mul(beta, c0);", "return c0;", "beta ignored when alpha = 0"),
    ("dd_oracle.c", "c = dd_add(c, dd_mul(beta, c0));", "c = dd_add(c, dd_mul(alpha, c0));",
     "alpha used for beta"),
    ("dd_oracle.c", "int64_t i, lo_i = upper ? 0 : j, hi_i = upper ? j : n - 1;",
     "int64_t i, lo_i = upper ? j : 0, hi_i = upper ? n - 1 : j;", "wrong Rsyrk triangle"),
    ("dd_oracle.c", "tb = !ta;\n#pragma omp parallel for schedule(dynamic, 1)",
     "tb = ta;\n#pragma omp parallel for schedule(dynamic, 1)", "Rsyrk without transpose"),
    ("dd_oracle.c", "int64_t nrowa = nota ? m : k;", "int64_t nrowa = nota ? k : m;",
     "wrong lda check"),
    ("dd_oracle.c", "if (ldc < imax(1, m)) return 13;", "if (ldc < imax(1, m)) return 12;",
     "wrong error code"),
    ("dd_oracle.c",
     "if (m == 0 || n == 0 || ((is_zero(alpha) || k == 0) && is_one(beta))) return 0;\n    ta",
     "if (m == 0 || n == 0 || ((is_zero(alpha) || k == 0) && is_zero(beta))) return 0;\n    ta",
     "wrong quick return"),
    ("dd_oracle.c", "if (!is_zero(beta)) { c0.hi = Ch[i + j * ldc]; c0.lo = Cl[i + j * ldc]; }\n"
     "            c = entry(ta, tb, i, j, k, alpha, Ah, Al, lda, Bh, Bl, ldb, beta, c0);",
     "c0.hi = Ch[i + j * ldc]; c0.lo = Cl[i + j * ldc];\n"
     "            c = entry(ta, tb, i, j, k, alpha, Ah, Al, lda, Bh, Bl, ldb, beta, c0);"
     "\n            if (is_zero(beta)) { c.hi += 0.0 * c0.hi; c.lo += 0.0 * c0.lo; }",
     "C read when beta = 0"),
    ("ozaki_oracle.c", "int shift = (t == 0) ? wfirst : w;", "int shift = w;",
     "first digit too wide"),
    ("ozaki_oracle.c", "y = two_sum(zh - q, zl);", "y.hi = zh - q; y.lo = 0.0;",
     "remainder drops the low part"),
    ("ozaki_oracle.c", "ldexp((double)x, -(2 * wfirst + w * (d - 2)))",
     "ldexp((double)x, -(2 * wfirst + w * (d - 1)))", "wrong anti-diagonal weight"),
    ("ozaki_oracle.c", "p.hi = ldexp(p.hi, ea[i] + eb[j]);", "p.hi = ldexp(p.hi, ea[i]);",
     "column scale dropped"),
    ("ozaki_oracle.c", "if (*q > qmax) {", "if (0) {", "digits not carried into int8's range"),
    ("ozaki_oracle.c", "digits[((int64_t)(t - 1) * rows + r) * k + l] += 1;",
     "digits[((int64_t)(t - 1) * rows + r) * k + l] += 0;", "carry lost"),
    ("ozaki_oracle.c", "*q -= (int32_t)1 << w;", "*q -= (int32_t)1 << (w - 1);",
     "carry of the wrong weight"),
    ("ozaki_oracle.c", "for (t = nslices - 1; t >= 1; --t) {", "for (t = 1; t < nslices; ++t) {",
     "carries propagated in the wrong order"),
    ("cdd_oracle.c", "r.re = dd_add(dd_mul(x.re, y.re), dd_neg(dd_mul(x.im, y.im)));",
     "r.re = dd_add(dd_mul(x.re, y.re), dd_mul(x.im, y.im));", "complex product: sign of bd"),
    ("cdd_oracle.c", "r.im = dd_add(dd_mul(x.re, y.im), dd_mul(x.im, y.re));",
     "r.im = dd_add(dd_mul(x.re, y.im), dd_mul(x.im, y.im));",
     "complex product: wrong cross term"),
    ("cdd_oracle.c", "if (mode == 2) v.im = dd_neg(v.im);", "",
     "conjugate transpose without conjugation"),
    ("cdd_oracle.c", "if (mode == 2) v.im = dd_neg(v.im);", "if (mode >= 1) v.im = dd_neg(v.im);",
     "plain transpose conjugated"),
    ("cdd_oracle.c", "c = c_add(c, c_mul(beta, c0));", "c = c_add(c, c_mul(alpha, c0));",
     "complex: alpha used for beta"),
    ("cdd_oracle.c", "return x.re.hi == 1.0 && x.re.lo == 0.0 && dd_is_zero(x.im);",
     "return x.re.hi == 1.0 && x.re.lo == 0.0;", "complex quick return ignores Im(beta)"),
    ("cdd_oracle.c", "if (ldb < c_imax(1, nrowb)) return 10;", "if (ldb < c_imax(1, nrowa)) return 10;",
     "complex: wrong ldb check"),
    ("cdd_oracle.c", "for (l = 0; l < k; ++l)\n", "for (l = 1; l < k; ++l)\n",
     "complex: dropped first term"),
    ("dd_ops.h", "double tl = d / y.hi;", "double tl = 0.0 * d / y.hi;",
     "dd division without the remainder correction"),
    ("dd_ops.h", "double dl = x.lo - r.lo;", "double dl = x.lo + r.lo;",
     "sign error in the division remainder"),
    ("dd_ops.h", "double r2 = x.lo + r1;", "double r2 = r1;", "square root ignores the low part"),
    ("dd_ops.h", "double sl = r2 / (2.0 * sh);", "double sl = r2 / sh;",
     "square root correction not halved"),
    ("potrf_oracle.c", "d = dd_add(d, p_neg(dd_mul(v, v)));", "d = dd_add(d, dd_mul(v, v));",
     "Cholesky: diagonal update added"),
    ("potrf_oracle.c", "odd a = {Ah[oi], Al[oi]}, b = {Ah[oj], Al[oj]};",
     "odd a = {Ah[oi], Al[oi]}, b = {Ah[oi], Al[oi]};", "Cholesky: wrong row in the update"),
    ("potrf_oracle.c", "return j + 1;", "return j;", "Cholesky: info off by one"),
    ("potrf_oracle.c", "if (!(d.hi > 0.0)) {", "if (d.hi < 0.0) {",
     "Cholesky: zero or NaN pivot accepted"),
    ("potrf_oracle.c", "return upper ? (l + i * lda) : (i + l * lda);",
     "return (i + l * lda);", "Cholesky: upper written as lower"),
    ("potrf_oracle.c", "acc = dd_div(acc, ljj);", "acc = dd_div(acc, d);",
     "Cholesky: divided by the pivot instead of its root"),
    ("qd_oracle.c", "if (rem > half || (rem == half && (sticky || (mant & 1)))) mant += 1;",
     "if (rem > half && 0) mant += 1;", "qd rounding truncates"),
    ("qd_oracle.c", "if (rem > half || (rem == half && (sticky || (mant & 1)))) mant += 1;",
     "if (rem >= half) mant += 1;", "qd rounding ties away from zero"),
    ("qd_oracle.c", "    qacc_add(acc, e3);\n", "", "qd: last part of a triple product dropped"),
    ("qd_oracle.c", "int64_t c = a->d[i] >> 32;     /* arithmetic shift: floor division */",
     "int64_t c = a->d[i] >> 31;", "qd accumulator: wrong carry"),
    ("qd_oracle.c", "for (p = 0; p < 4; ++p) qacc_add2(&acc, beta[r], C[p][o]);",
     "for (p = 0; p < 4; ++p) qacc_add2(&acc, beta[0], C[p][o]);", "qd: beta's low parts ignored"),
    ("qd_oracle.c", "if (alpha[r] == 0.0) continue;", "if (r > 0) continue;",
     "qd: alpha's low parts ignored"),
    ("qd_oracle.c", "((q_zero(alpha) || k == 0) && q_one(beta))) return 0;",
     "((q_zero(alpha) || k == 0) && q_zero(beta))) return 0;", "qd: wrong quick return"),
    ("qd_oracle.c", "    if (neg) {                          /* two's complement negate",
     "    if (0) {                          /* two's complement negate", "qd: sign lost in rounding"),
]

CHECKS = [
    pins.check_worked_example,
    pins.check_primitives,
    lambda lib: pins.check_exact_gemm(lib, seeds=[0, 1]),
    lambda lib: pins.check_exact_syrk(lib, seeds=[0]),
    pins.check_info_codes,
    pins.check_identities,
    lambda lib: pins.check_ozaki_split_exact(lib),
    pins.check_ozaki_gemm_exact,
    pins.check_cgemm_worked_example,
    lambda lib: pins.check_exact_cgemm(lib, seeds=[0]),
    pins.check_cgemm_identities,
    pins.check_cgemm_info_codes,
    pins.check_div_sqrt,
    pins.check_potrf_exact_integer,
    lambda lib: pins.check_potrf_residual(lib, sizes=(3, 6)),
    pins.check_potrf_transpose_and_info,
    pins.check_qd_round,
    lambda lib: pins.check_qgemm_exact(lib, seeds=[0]),
    pins.check_qgemm_semantics,
]


def _caught(lib):
    for chk in CHECKS:
        try:
            chk(lib)
        except (AssertionError, ValueError):
            return True
    return False


@pytest.mark.parametrize("fname,orig,mut,what", MUTANTS, ids=[m[3] for m in MUTANTS])
def test_mutant_is_caught(fname, orig, mut, what):
    tmp = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        for f in SOURCES + ["dd_ops.h"]:
            shutil.copy(os.path.join(SRC, f), tmp)
        path = os.path.join(tmp, fname)
        text = open(path).read()
        assert text.count(orig) == 1, f"mutation anchor not found once: {orig!r}"
        open(path, "w").write(text.replace(orig, mut))
        so = obuild.build(out=os.path.join(tmp, "libmut.so"),
                          sources=SOURCES, cwd=tmp,
                          extra=["-I", tmp])
        lib = oracle.load(so)
        assert _caught(lib), f"planted mistake not caught: {what}"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def test_unmutated_copy_passes():
    """Control: the same harness on an unmodified copy passes every check."""
    tmp = tempfile.mkdtemp(prefix="oracle_ctl_")
    try:
        for f in SOURCES + ["dd_ops.h"]:
            shutil.copy(os.path.join(SRC, f), tmp)
        so = obuild.build(out=os.path.join(tmp, "libctl.so"),
                          sources=SOURCES, cwd=tmp,
                          extra=["-I", tmp])
        assert not _caught(oracle.load(so))
    finally:
        shutil.rmtree(tmp, ignore_errors=True)

/*
 * cdd_oracle.c -- CPU oracle for the complex double-double Cgemm.
 *
 * TEST INFRASTRUCTURE ONLY.  Like dd_oracle.c, this is the slow,
 * obviously-correct reference the GPU library is checked against; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it, and it shares no code with the GPU library.
 *
 * What it computes (MPLAPACK 2.0.1 manual, section "How to use reference
 * MPBLAS", the Cgemm part: Cgemm is ZGEMM's calling convention with complex
 * multiple-precision scalars and column-major arrays):
 *
 *   C <- alpha * op(A) * op(B) + beta * C,
 *   op(X) = X ('N'), X^T ('T') or conj(X)^T ('C').
 *
 * A complex dd value is a pair (re, im) of dd values.  Complex arithmetic is
 * the textbook definition on top of the dd operations of dd_ops.h:
 *   (a + ib) (c + id) = (ac - bd) + i (ad + bc),
 * each real product a dd multiply (DWTimesDW3), each sum a dd add
 * (AccurateDWPlusDW); the terms of the dot product are summed in increasing
 * l, alpha is applied once to the finished sum, then beta * C is added, the
 * same order as the real oracle.
 *
 * Argument checks and quick returns follow the BLAS ZGEMM reference: the
 * return value is 0 or the 1-based position of the first bad argument
 * (1 transa, 2 transb, 3 m, 4 n, 5 k, 8 lda, 10 ldb, 13 ldc), and nothing
 * is written when it is non-zero.
 *
 * Storage: every complex matrix is four binary64 planes (re.hi, re.lo,
 * im.hi, im.lo), each column-major with the same leading dimension.
 */
#include <stdint.h>
#include <stddef.h>

#include "dd_ops.h"

typedef struct { odd re, im; } ocd;

/* the four planes of one complex dd matrix */
typedef struct { const double *rh, *rl, *ih, *il; } cplanes_in;

static int c_lsame(const char *s, char ref)
{
    char c;
    if (s == NULL) return 0;
    c = s[0];
    if (c >= 'a' && c <= 'z') c = (char)(c - 'a' + 'A');
    return c == ref;
}

static int64_t c_imax(int64_t a, int64_t b) { return a > b ? a : b; }

static int dd_is_zero(odd x) { return x.hi == 0.0 && x.lo == 0.0; }
static int c_is_zero(ocd x) { return dd_is_zero(x.re) && dd_is_zero(x.im); }
static int c_is_one(ocd x)
{
    return x.re.hi == 1.0 && x.re.lo == 0.0 && dd_is_zero(x.im);
}

static odd dd_neg(odd x) { odd r; r.hi = -x.hi; r.lo = -x.lo; return r; }

static ocd c_add(ocd x, ocd y)
{
    ocd r;
    r.re = dd_add(x.re, y.re);
    r.im = dd_add(x.im, y.im);
    return r;
}

static ocd c_mul(ocd x, ocd y)
{
    ocd r;
    r.re = dd_add(dd_mul(x.re, y.re), dd_neg(dd_mul(x.im, y.im)));
    r.im = dd_add(dd_mul(x.re, y.im), dd_mul(x.im, y.re));
    return r;
}

/* op(X)(r, c) with mode 0 = N, 1 = T, 2 = C (conjugate transpose) */
static ocd c_load(cplanes_in x, int64_t ld, int mode, int64_t r, int64_t c)
{
    ocd v;
    int64_t idx = mode ? (c + r * ld) : (r + c * ld);
    v.re.hi = x.rh[idx]; v.re.lo = x.rl[idx];
    v.im.hi = x.ih[idx]; v.im.lo = x.il[idx];
    if (mode == 2) v.im = dd_neg(v.im);
    return v;
}

static int c_check(const char *transa, const char *transb, int64_t m, int64_t n, int64_t k,
                   int64_t lda, int64_t ldb, int64_t ldc)
{
    int nota = c_lsame(transa, 'N'), notb = c_lsame(transb, 'N');
    int64_t nrowa = nota ? m : k;
    int64_t nrowb = notb ? k : n;
    if (!nota && !c_lsame(transa, 'T') && !c_lsame(transa, 'C')) return 1;
    if (!notb && !c_lsame(transb, 'T') && !c_lsame(transb, 'C')) return 2;
    if (m < 0) return 3;
    if (n < 0) return 4;
    if (k < 0) return 5;
    if (lda < c_imax(1, nrowa)) return 8;
    if (ldb < c_imax(1, nrowb)) return 10;
    if (ldc < c_imax(1, m)) return 13;
    return 0;
}

static int c_mode(const char *t)
{
    if (c_lsame(t, 'N')) return 0;
    if (c_lsame(t, 'T')) return 1;
    return 2;
}

int oracle_Cgemm(const char *transa, const char *transb, int64_t m, int64_t n, int64_t k,
                 const double *alpha4, const double *Arh, const double *Arl, const double *Aih,
                 const double *Ail, int64_t lda, const double *Brh, const double *Brl,
                 const double *Bih, const double *Bil, int64_t ldb, const double *beta4,
                 double *Crh, double *Crl, double *Cih, double *Cil, int64_t ldc)
{
    int info = c_check(transa, transb, m, n, k, lda, ldb, ldc);
    int ma, mb;
    int64_t j;
    ocd alpha, beta;
    cplanes_in A, B;
    if (info) return info;
    alpha.re.hi = alpha4[0]; alpha.re.lo = alpha4[1];
    alpha.im.hi = alpha4[2]; alpha.im.lo = alpha4[3];
    beta.re.hi = beta4[0]; beta.re.lo = beta4[1];
    beta.im.hi = beta4[2]; beta.im.lo = beta4[3];
    if (m == 0 || n == 0 || ((c_is_zero(alpha) || k == 0) && c_is_one(beta))) return 0;
    ma = c_mode(transa);
    mb = c_mode(transb);
    A.rh = Arh; A.rl = Arl; A.ih = Aih; A.il = Ail;
    B.rh = Brh; B.rl = Brl; B.ih = Bih; B.il = Bil;
#pragma omp parallel for schedule(dynamic, 1)
    for (j = 0; j < n; ++j) {
        int64_t i, l;
        for (i = 0; i < m; ++i) {
            const int64_t o = i + j * ldc;
            ocd c0, c, acc;
            c0.re.hi = c0.re.lo = c0.im.hi = c0.im.lo = 0.0;
            if (!c_is_zero(beta)) {
                c0.re.hi = Crh[o]; c0.re.lo = Crl[o];
                c0.im.hi = Cih[o]; c0.im.lo = Cil[o];
            }
            if (c_is_zero(alpha) || k == 0) {
                if (c_is_zero(beta)) c = c0;            /* (+0, +0) */
                else c = c_mul(beta, c0);
            } else {
                acc.re.hi = acc.re.lo = acc.im.hi = acc.im.lo = 0.0;
                for (l = 0; l < k; ++l)
                    acc = c_add(acc, c_mul(c_load(A, lda, ma, i, l), c_load(B, ldb, mb, l, j)));
                c = c_mul(alpha, acc);
                if (!c_is_zero(beta)) c = c_add(c, c_mul(beta, c0));
            }
            Crh[o] = c.re.hi; Crl[o] = c.re.lo;
            Cih[o] = c.im.hi; Cil[o] = c.im.lo;
        }
    }
    return 0;
}

/*
 * dd_oracle.c -- CPU oracle for the double-double (dd) Rgemm / Rsyrk path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header or constant with the GPU library.
 *
 * What it computes (MPLAPACK 2.0.1 manual, section "How to use reference
 * MPBLAS": Rgemm follows the DGEMM calling convention, column-major
 * one-dimensional arrays with leading dimensions; Table "mpblasroutines"
 * lists Rgemm and Rsyrk as the level-3 routines):
 *
 *   Rgemm:  C <- alpha * op(A) * op(B) + beta * C,   op(X) = X or X^T
 *   Rsyrk:  C <- alpha * A * A^T + beta * C   (trans = 'N')
 *           C <- alpha * A^T * A + beta * C   (trans = 'T' or 'C')
 *           on the uplo triangle of C only (diagonal included).
 *
 * Number format (section "Supported Floating point formats"): a dd value is
 * the unevaluated sum hi + lo of two binary64 numbers, built from the
 * error-free transformations of Knuth (TwoSum) and Dekker (exact product);
 * about 32 decimal digits, epsilon 2^-104 (Table "rlamch_dd").  The manual
 * does not say which dd add/mul variants QD uses, so this oracle takes the
 * published algorithms with proven error bounds:
 *   - TwoSum (Knuth), FastTwoSum (Dekker), TwoProd via fused multiply-add;
 *   - dd + dd: "AccurateDWPlusDW" (Joldes, Muller, Popescu 2017), relative
 *     error <= 3u^2 + 13u^3, u = 2^-53;
 *   - dd * dd: "DWTimesDW3" (same paper), relative error <= 4u^2.
 * The loop is the plain definition: for every referenced (i, j) the terms
 * op(A)(i,l)*op(B)(l,j) are formed as dd products and summed in increasing
 * l; alpha is applied once to the finished sum, then beta*C is added.
 *
 * Argument checking and quick returns follow the BLAS reference routines
 * (the manual's MPBLAS quality-assurance section requires the error codes to
 * equal xerbla's): the return value is 0 or the 1-based position of the
 * first invalid argument; nothing is written when it is non-zero.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no FMA contraction, so every
 * rounding step is the one written here).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#include "dd_ops.h"

/* ---- BLAS flag handling (lsame: first character, case-insensitive) ---- */

static int lsame(const char *s, char ref)
{
    char c;
    if (s == NULL) return 0;
    c = s[0];
    if (c >= 'a' && c <= 'z') c = (char)(c - 'a' + 'A');
    return c == ref;
}

static int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }

static int is_zero(odd x) { return x.hi == 0.0 && x.lo == 0.0; }
static int is_one(odd x)  { return x.hi == 1.0 && x.lo == 0.0; }

/* ---- exported primitives (for the tests that pin them) ----------------- */

void oracle_two_sum(double a, double b, double *s, double *e)
{ odd r = two_sum(a, b); *s = r.hi; *e = r.lo; }

void oracle_two_prod(double a, double b, double *p, double *e)
{ odd r = two_prod(a, b); *p = r.hi; *e = r.lo; }

void oracle_dd_add(double xh, double xl, double yh, double yl, double *zh, double *zl)
{
    odd x = {xh, xl}, y = {yh, yl};
    odd z = dd_add(x, y);
    *zh = z.hi; *zl = z.lo;
}

void oracle_dd_mul(double xh, double xl, double yh, double yl, double *zh, double *zl)
{
    odd x = {xh, xl}, y = {yh, yl};
    odd z = dd_mul(x, y);
    *zh = z.hi; *zl = z.lo;
}

/* ---- one output entry --------------------------------------------------- */

/* op(A)(i,l): A[i + l*lda] when not transposed, A[l + i*lda] when transposed. */
static inline odd load_op(const double *hi, const double *lo, int64_t ld,
                          int trans, int64_t r, int64_t c)
{
    odd v;
    int64_t idx = trans ? (c + r * ld) : (r + c * ld);
    v.hi = hi[idx]; v.lo = lo[idx];
    return v;
}

/* The value of entry (i, j) after the update, given its previous value c0. */
static odd entry(int ta, int tb, int64_t i, int64_t j, int64_t k, odd alpha,
                 const double *Ah, const double *Al, int64_t lda,
                 const double *Bh, const double *Bl, int64_t ldb,
                 odd beta, odd c0)
{
    odd c, acc;
    int64_t l;
    if (is_zero(alpha) || k == 0) {
        if (is_zero(beta)) { c.hi = 0.0; c.lo = 0.0; return c; }
        return dd_mul(beta, c0);
    }
    acc.hi = 0.0; acc.lo = 0.0;
    for (l = 0; l < k; ++l) {
        odd a = load_op(Ah, Al, lda, ta, i, l);
        odd b = load_op(Bh, Bl, ldb, tb, l, j);
        acc = dd_add(acc, dd_mul(a, b));
    }
    c = dd_mul(alpha, acc);
    if (!is_zero(beta))
        c = dd_add(c, dd_mul(beta, c0));
    return c;
}

/* ---- Rgemm -------------------------------------------------------------- */

static int check_gemm(const char *transa, const char *transb, int64_t m, int64_t n,
                      int64_t k, int64_t lda, int64_t ldb, int64_t ldc)
{
    int nota = lsame(transa, 'N'), notb = lsame(transb, 'N');
    int64_t nrowa = nota ? m : k;
    int64_t nrowb = notb ? k : n;
    if (!nota && !lsame(transa, 'T') && !lsame(transa, 'C')) return 1;
    if (!notb && !lsame(transb, 'T') && !lsame(transb, 'C')) return 2;
    if (m < 0) return 3;
    if (n < 0) return 4;
    if (k < 0) return 5;
    if (lda < imax(1, nrowa)) return 8;
    if (ldb < imax(1, nrowb)) return 10;
    if (ldc < imax(1, m)) return 13;
    return 0;
}

int oracle_Rgemm(const char *transa, const char *transb, int64_t m, int64_t n, int64_t k,
                 odd alpha, const double *Ah, const double *Al, int64_t lda,
                 const double *Bh, const double *Bl, int64_t ldb,
                 odd beta, double *Ch, double *Cl, int64_t ldc)
{
    int info = check_gemm(transa, transb, m, n, k, lda, ldb, ldc);
    int ta, tb;
    int64_t j;
    if (info) return info;
    if (m == 0 || n == 0 || ((is_zero(alpha) || k == 0) && is_one(beta))) return 0;
    ta = !lsame(transa, 'N');
    tb = !lsame(transb, 'N');
#pragma omp parallel for schedule(dynamic, 1)
    for (j = 0; j < n; ++j) {
        int64_t i;
        for (i = 0; i < m; ++i) {
            odd c0 = {0.0, 0.0};
            odd c;
            if (!is_zero(beta)) { c0.hi = Ch[i + j * ldc]; c0.lo = Cl[i + j * ldc]; }
            c = entry(ta, tb, i, j, k, alpha, Ah, Al, lda, Bh, Bl, ldb, beta, c0);
            Ch[i + j * ldc] = c.hi;
            Cl[i + j * ldc] = c.lo;
        }
    }
    return 0;
}

/* Entries (ii[t], jj[t]) of the Rgemm result, written to out_hi/out_lo[t];
 * C is read (when beta != 0) but never written.  Used to check very large
 * products on a sample of their entries. */
int oracle_Rgemm_entries(const char *transa, const char *transb, int64_t m, int64_t n,
                         int64_t k, odd alpha, const double *Ah, const double *Al,
                         int64_t lda, const double *Bh, const double *Bl, int64_t ldb,
                         odd beta, const double *Ch, const double *Cl, int64_t ldc,
                         int64_t count, const int64_t *ii, const int64_t *jj,
                         double *out_hi, double *out_lo)
{
    int info = check_gemm(transa, transb, m, n, k, lda, ldb, ldc);
    int ta, tb;
    int64_t t;
    if (info) return info;
    ta = !lsame(transa, 'N');
    tb = !lsame(transb, 'N');
    for (t = 0; t < count; ++t)
        if (ii[t] < 0 || ii[t] >= m || jj[t] < 0 || jj[t] >= n) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (t = 0; t < count; ++t) {
        int64_t i = ii[t], j = jj[t];
        odd c0 = {0.0, 0.0};
        odd c;
        if (!is_zero(beta)) { c0.hi = Ch[i + j * ldc]; c0.lo = Cl[i + j * ldc]; }
        if (is_zero(alpha) || k == 0) {
            if (is_one(beta)) c = c0;
            else c = entry(ta, tb, i, j, k, alpha, Ah, Al, lda, Bh, Bl, ldb, beta, c0);
        } else {
            c = entry(ta, tb, i, j, k, alpha, Ah, Al, lda, Bh, Bl, ldb, beta, c0);
        }
        out_hi[t] = c.hi;
        out_lo[t] = c.lo;
    }
    return 0;
}

/* ---- Rsyrk -------------------------------------------------------------- */

static int check_syrk(const char *uplo, const char *trans, int64_t n, int64_t k,
                      int64_t lda, int64_t ldc)
{
    int upper = lsame(uplo, 'U');
    int64_t nrowa = lsame(trans, 'N') ? n : k;
    if (!upper && !lsame(uplo, 'L')) return 1;
    if (!lsame(trans, 'N') && !lsame(trans, 'T') && !lsame(trans, 'C')) return 2;
    if (n < 0) return 3;
    if (k < 0) return 4;
    if (lda < imax(1, nrowa)) return 7;
    if (ldc < imax(1, n)) return 10;
    return 0;
}

/* Rsyrk is Rgemm with op(B) = op(A)^T taken from the same array:
 * trans = 'N': op(A)(i,l) = A[i + l*lda], op(B)(l,j) = A[j + l*lda];
 * trans = 'T': op(A)(i,l) = A[l + i*lda], op(B)(l,j) = A[l + j*lda]. */
int oracle_Rsyrk(const char *uplo, const char *trans, int64_t n, int64_t k,
                 odd alpha, const double *Ah, const double *Al, int64_t lda,
                 odd beta, double *Ch, double *Cl, int64_t ldc)
{
    int info = check_syrk(uplo, trans, n, k, lda, ldc);
    int upper, ta, tb;
    int64_t j;
    if (info) return info;
    if (n == 0 || ((is_zero(alpha) || k == 0) && is_one(beta))) return 0;
    upper = lsame(uplo, 'U');
    ta = !lsame(trans, 'N');
    tb = !ta;
#pragma omp parallel for schedule(dynamic, 1)
    for (j = 0; j < n; ++j) {
        int64_t i, lo_i = upper ? 0 : j, hi_i = upper ? j : n - 1;
        for (i = lo_i; i <= hi_i; ++i) {
            odd c0 = {0.0, 0.0};
            odd c;
            if (!is_zero(beta)) { c0.hi = Ch[i + j * ldc]; c0.lo = Cl[i + j * ldc]; }
            c = entry(ta, tb, i, j, k, alpha, Ah, Al, lda, Ah, Al, lda, beta, c0);
            Ch[i + j * ldc] = c.hi;
            Cl[i + j * ldc] = c.lo;
        }
    }
    return 0;
}

/* Sampled Rsyrk entries; every (ii[t], jj[t]) must lie in the uplo triangle. */
int oracle_Rsyrk_entries(const char *uplo, const char *trans, int64_t n, int64_t k,
                         odd alpha, const double *Ah, const double *Al, int64_t lda,
                         odd beta, const double *Ch, const double *Cl, int64_t ldc,
                         int64_t count, const int64_t *ii, const int64_t *jj,
                         double *out_hi, double *out_lo)
{
    int info = check_syrk(uplo, trans, n, k, lda, ldc);
    int upper, ta, tb;
    int64_t t;
    if (info) return info;
    upper = lsame(uplo, 'U');
    ta = !lsame(trans, 'N');
    tb = !ta;
    for (t = 0; t < count; ++t) {
        if (ii[t] < 0 || ii[t] >= n || jj[t] < 0 || jj[t] >= n) return -1;
        if (upper ? (ii[t] > jj[t]) : (ii[t] < jj[t])) return -1;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (t = 0; t < count; ++t) {
        int64_t i = ii[t], j = jj[t];
        odd c0 = {0.0, 0.0};
        odd c;
        if (!is_zero(beta)) { c0.hi = Ch[i + j * ldc]; c0.lo = Cl[i + j * ldc]; }
        if ((is_zero(alpha) || k == 0) && is_one(beta)) c = c0;
        else c = entry(ta, tb, i, j, k, alpha, Ah, Al, lda, Ah, Al, lda, beta, c0);
        out_hi[t] = c.hi;
        out_lo[t] = c.lo;
    }
    return 0;
}

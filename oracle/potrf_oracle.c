/*
 * potrf_oracle.c -- CPU oracle for the dd Cholesky factorisation Rpotrf.
 *
 * TEST INFRASTRUCTURE ONLY (like dd_oracle.c): the slow, obviously-correct
 * reference the GPU library is checked against; it shares no code with the
 * GPU library.
 *
 * What it computes (MPLAPACK 2.0.1 manual: Rpotrf is LAPACK's DPOTRF on
 * multiple-precision values, listed among the MPLAPACK routines and timed in
 * the section on Rpotrf performance; the interior-point solvers the manual
 * motivates MPLAPACK with factor their Schur complement matrices this way):
 * for a symmetric positive definite A (only the uplo triangle is referenced)
 *
 *   uplo = 'L':  A = L L^T,  L lower triangular, written over the lower triangle;
 *   uplo = 'U':  A = U^T U,  U upper triangular, written over the upper triangle.
 *
 * The plain definition, column by column (Cholesky-Crout), in the lower view
 * L(i, l) (= U(l, i) for uplo 'U'):
 *   d = A(j,j) - sum_{l<j} L(j,l)^2;  d <= 0 or NaN -> info = j+1, A(j,j) = d, stop;
 *   L(j,j) = sqrt(d);
 *   L(i,j) = (A(i,j) - sum_{l<j} L(i,l) L(j,l)) / L(j,j),  i > j,
 * every sum formed by subtracting the dd products in increasing l with the
 * dd operations of dd_ops.h (products DWTimesDW3, sums AccurateDWPlusDW,
 * quotient DWDivDW2, square root with one remainder correction).
 *
 * Return value: LAPACK's info -- 0; -1 (uplo), -2 (n < 0), -4 (lda <
 * max(1, n)) with nothing written; or j+1 > 0 when the leading minor of
 * order j+1 is not positive definite.  The opposite triangle and the rows
 * below n are never read or written.
 */
#include <stdint.h>
#include <stddef.h>

#include "dd_ops.h"

static int p_lsame(const char *s, char ref)
{
    char c;
    if (s == NULL) return 0;
    c = s[0];
    if (c >= 'a' && c <= 'z') c = (char)(c - 'a' + 'A');
    return c == ref;
}

static odd p_neg(odd x) { odd r; r.hi = -x.hi; r.lo = -x.lo; return r; }

/* storage index of L(i, l) (i >= l) in the lower view */
static inline int64_t lidx(int upper, int64_t i, int64_t l, int64_t lda)
{
    return upper ? (l + i * lda) : (i + l * lda);
}

void oracle_dd_div(double xh, double xl, double yh, double yl, double *zh, double *zl)
{
    odd x = {xh, xl}, y = {yh, yl};
    odd z = dd_div(x, y);
    *zh = z.hi; *zl = z.lo;
}

void oracle_dd_sqrt(double xh, double xl, double *zh, double *zl)
{
    odd x = {xh, xl};
    odd z = dd_sqrt(x);
    *zh = z.hi; *zl = z.lo;
}

int64_t oracle_Rpotrf(const char *uplo, int64_t n, double *Ah, double *Al, int64_t lda)
{
    int upper = p_lsame(uplo, 'U');
    int64_t j;
    if (!upper && !p_lsame(uplo, 'L')) return -1;
    if (n < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -4;
    for (j = 0; j < n; ++j) {
        int64_t l, i;
        const int64_t jj = lidx(upper, j, j, lda);
        odd d, ljj;
        d.hi = Ah[jj]; d.lo = Al[jj];
        for (l = 0; l < j; ++l) {
            const int64_t o = lidx(upper, j, l, lda);
            odd v = {Ah[o], Al[o]};
            d = dd_add(d, p_neg(dd_mul(v, v)));
        }
        if (!(d.hi > 0.0)) {
            Ah[jj] = d.hi; Al[jj] = d.lo;
            return j + 1;
        }
        ljj = dd_sqrt(d);
        Ah[jj] = ljj.hi; Al[jj] = ljj.lo;
#pragma omp parallel for schedule(static)
        for (i = j + 1; i < n; ++i) {
            int64_t q;
            const int64_t ij = lidx(upper, i, j, lda);
            odd acc = {Ah[ij], Al[ij]};
            for (q = 0; q < j; ++q) {
                const int64_t oi = lidx(upper, i, q, lda), oj = lidx(upper, j, q, lda);
                odd a = {Ah[oi], Al[oi]}, b = {Ah[oj], Al[oj]};
                acc = dd_add(acc, p_neg(dd_mul(a, b)));
            }
            acc = dd_div(acc, ljj);
            Ah[ij] = acc.hi; Al[ij] = acc.lo;
        }
    }
    return 0;
}

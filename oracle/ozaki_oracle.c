/*
 * ozaki_oracle.c -- CPU oracle for the Ozaki-style split form of dd Rgemm.
 *
 * TEST INFRASTRUCTURE ONLY (see dd_oracle.c).  Shares no code with the GPU
 * library.
 *
 * The manual itself contains no split method; this follows the error-free
 * splitting of a matrix product (Ozaki, Ogita, Oishi, Rump, "Error-free
 * transformations of matrix multiplication by using fast routines of matrix
 * multiplication and its applications", Numer. Algorithms 2012) and its
 * integer-unit form (Ootomo, Ozaki, Yokota, "DGEMM on integer matrix
 * multiplication unit", IJHPCA 2024), applied to dd operands:
 *
 *  1. Scale.  For row r of the row operand (a row of op(A), or a column of
 *     op(B)), sigma_r is the exponent with max_l |x_rl.hi| = f * 2^sigma_r,
 *     f in [1/2, 1) (frexp); then |x_rl| < 2^sigma_r for a normalised dd.
 *     An all-zero row gets sigma_r = 0 and zero digits.
 *  2. Slice.  y_0 = x * 2^-sigma in (-1, 1) (exact).  Digit t = 1..s:
 *     z = y_{t-1} * 2^{w_t} (exact), q_t = nearest integer to z.hi (ties to
 *     even), y_t = TwoSum(z.hi - q_t, z.lo).  w_1 = wfirst, w_t = w after.
 *     Then x = 2^sigma * (sum_t q_t 2^-W_t + y_s 2^-W_s), W_t = wfirst +
 *     w (t-1), and |q_t| <= 2^{wfirst} (first digit) and <= 2^{w-1} (rest).
 *  2b. Storage range.  When the digits are stored in a narrow integer type
 *     whose largest value is qmax (int8: 127), every digit after the first
 *     that exceeds qmax is lowered by 2^w and the digit before it raised by
 *     one, from the last digit to the second.  The represented value does not
 *     change (2^w units of digit t make one unit of digit t-1).  Rounded
 *     digits lie in [-2^{w-1}, 2^{w-1}] and a digit receives a carry of at
 *     most one, so with qmax = 2^{w-1} - 1 every later digit ends in
 *     [-2^{w-1}, 2^{w-1} - 1] and the first in [-2^wfirst, 2^wfirst + 1].
 *     INT8 slices: wfirst = 6 and w = 8 (digits in [-128, 127]) while
 *     nslices * k < 2^17, else w = 7 (|q_t| <= 64, no carry ever needed)
 *     while nslices * k < 2^19: every anti-diagonal sum of at most
 *     nslices * k digit products, each at most 2^{2w-2} in magnitude, then
 *     stays below 2^31.
 *  3. Products.  For every anti-diagonal d = t + u, 2 <= d <= s + 1:
 *     X_d = sum_{t+u=d} Q_t Q'_u^T, computed exactly (integers).
 *  4. Recombine.  P_ij = sum_d X_d(i,j) 2^-(2 wfirst + w (d-2)), summed in dd
 *     from the smallest weight (d = s + 1) to the largest (d = 2) with
 *     DWPlusFP; then P_ij * 2^(sigma_i + tau_j) (exact), and the same
 *     alpha/beta update as the plain Rgemm: C = alpha*P + beta*C.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "dd_ops.h"

/* Element (r, l) of a row operand stored at p[r*sr + l*sl]. */
static inline odd at(const double *hi, const double *lo, int64_t sr, int64_t sl,
                     int64_t r, int64_t l)
{
    odd v;
    v.hi = hi[r * sr + l * sl];
    v.lo = lo[r * sr + l * sl];
    return v;
}

/* Scale exponents and digits of a rows x k row operand.
 * exps[r]: sigma_r.  digits[(t*rows + r)*k + l]: q_{t+1} of element (r, l).
 * qmax > 0: carry the digits after the first into [.., qmax] (step 2b);
 * qmax = 0: digits as rounded. */
int oracle_ozaki_split(int64_t rows, int64_t k, const double *hi, const double *lo,
                       int64_t sr, int64_t sl, int nslices, int wfirst, int w, int qmax,
                       int32_t *exps, int32_t *digits)
{
    int64_t r;
    if (rows < 0 || k < 0 || nslices < 1 || wfirst < 1 || w < 1) return -1;
#pragma omp parallel for schedule(static)
    for (r = 0; r < rows; ++r) {
        int64_t l;
        int t, e = 0;
        double mx = 0.0;
        for (l = 0; l < k; ++l) {
            double a = fabs(hi[r * sr + l * sl]);
            if (a > mx) mx = a;
        }
        if (mx != 0.0) frexp(mx, &e);
        exps[r] = e;
        for (l = 0; l < k; ++l) {
            odd y = at(hi, lo, sr, sl, r, l);
            if (mx == 0.0) { y.hi = 0.0; y.lo = 0.0; }
            y.hi = ldexp(y.hi, -e);
            y.lo = ldexp(y.lo, -e);
            for (t = 0; t < nslices; ++t) {
                int shift = (t == 0) ? wfirst : w;
                double zh = ldexp(y.hi, shift), zl = ldexp(y.lo, shift);
                double q = nearbyint(zh);   /* default rounding: ties to even */
                digits[((int64_t)t * rows + r) * k + l] = (int32_t)q;
                y = two_sum(zh - q, zl);
            }
            if (qmax > 0) {
                for (t = nslices - 1; t >= 1; --t) {
                    int32_t *q = &digits[((int64_t)t * rows + r) * k + l];
                    if (*q > qmax) {
                        *q -= (int32_t)1 << w;
                        digits[((int64_t)(t - 1) * rows + r) * k + l] += 1;
                    }
                }
            }
        }
    }
    return 0;
}

/* Full split-form product for the NN/NT/TN/TT cases:
 * C <- alpha * op(A) op(B) + beta * C with op(A), op(B) rebuilt from
 * nslices digits each.  Returns 0, or -1 on bad sizes / allocation failure.
 * Quick returns and the alpha == 0 / k == 0 cases match the plain routine. */
int oracle_ozaki_Rgemm(const char *transa, const char *transb, int64_t m, int64_t n,
                       int64_t k, odd alpha, const double *Ah, const double *Al,
                       int64_t lda, const double *Bh, const double *Bl, int64_t ldb,
                       odd beta, double *Ch, double *Cl, int64_t ldc,
                       int nslices, int wfirst, int w, int qmax)
{
    int ta = !(transa[0] == 'N' || transa[0] == 'n');
    int tb = !(transb[0] == 'N' || transb[0] == 'n');
    int32_t *ea, *eb, *qa, *qb;
    int64_t j;
    int alpha0 = (alpha.hi == 0.0 && alpha.lo == 0.0);
    int beta0 = (beta.hi == 0.0 && beta.lo == 0.0);
    int beta1 = (beta.hi == 1.0 && beta.lo == 0.0);
    if (m < 0 || n < 0 || k < 0 || nslices < 1) return -1;
    if (m == 0 || n == 0 || ((alpha0 || k == 0) && beta1)) return 0;
    if (alpha0 || k == 0) {
        for (j = 0; j < n; ++j) {
            int64_t i;
            for (i = 0; i < m; ++i) {
                odd c;
                if (beta0) { c.hi = 0.0; c.lo = 0.0; }
                else {
                    odd c0 = {Ch[i + j * ldc], Cl[i + j * ldc]};
                    c = dd_mul(beta, c0);
                }
                Ch[i + j * ldc] = c.hi;
                Cl[i + j * ldc] = c.lo;
            }
        }
        return 0;
    }
    ea = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    eb = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    qa = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nslices * m * k));
    qb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nslices * n * k));
    if (!ea || !eb || !qa || !qb) { free(ea); free(eb); free(qa); free(qb); return -1; }
    /* row operand of A: op(A)(i, l) */
    oracle_ozaki_split(m, k, Ah, Al, ta ? lda : 1, ta ? 1 : lda, nslices, wfirst, w, qmax, ea,
                       qa);
    /* row operand of B: op(B)(l, j) seen as element (j, l) */
    oracle_ozaki_split(n, k, Bh, Bl, tb ? 1 : ldb, tb ? ldb : 1, nslices, wfirst, w, qmax, eb,
                       qb);

#pragma omp parallel for schedule(dynamic, 1)
    for (j = 0; j < n; ++j) {
        int64_t i;
        for (i = 0; i < m; ++i) {
            odd p = {0.0, 0.0}, c;
            int d;
            for (d = nslices + 1; d >= 2; --d) {
                int64_t x = 0;
                int t;
                for (t = 1; t <= d - 1; ++t) {
                    int u = d - t;
                    const int32_t *ra, *rb;
                    int64_t l;
                    if (t > nslices || u > nslices) continue;
                    ra = qa + ((int64_t)(t - 1) * m + i) * k;
                    rb = qb + ((int64_t)(u - 1) * n + j) * k;
                    for (l = 0; l < k; ++l) x += (int64_t)ra[l] * (int64_t)rb[l];
                }
                p = dd_add_d(p, ldexp((double)x, -(2 * wfirst + w * (d - 2))));
            }
            p.hi = ldexp(p.hi, ea[i] + eb[j]);
            p.lo = ldexp(p.lo, ea[i] + eb[j]);
            c = dd_mul(alpha, p);
            if (!beta0) {
                odd c0 = {Ch[i + j * ldc], Cl[i + j * ldc]};
                c = dd_add(c, dd_mul(beta, c0));
            }
            Ch[i + j * ldc] = c.hi;
            Cl[i + j * ldc] = c.lo;
        }
    }
    free(ea); free(eb); free(qa); free(qb);
    return 0;
}

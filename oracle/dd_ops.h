/*
 * dd_ops.h -- double-double arithmetic of the CPU oracle (test
 * infrastructure only; never included by the GPU library).
 *
 * The dd format is the unevaluated sum hi + lo of two binary64 numbers
 * (manual, section "Supported Floating point formats": Knuth's and Dekker's
 * error-free algorithms, via the QD library).  The concrete add and multiply
 * are the published algorithms with proven bounds (Joldes, Muller, Popescu,
 * "Tight and rigorous error bounds for basic building blocks of double-word
 * arithmetic", ACM TOMS 2017), since the manual does not name QD's variants.
 * Compile with -ffp-contract=off.
 */
#ifndef DD_ORACLE_OPS_H
#define DD_ORACLE_OPS_H
#include <math.h>

typedef struct { double hi, lo; } odd;   /* oracle dd value */

/* Knuth's TwoSum: s = fl(a+b), e = (a+b) - s exactly, no branch. */
static inline odd two_sum(double a, double b)
{
    odd r;
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    r.hi = s; r.lo = e;
    return r;
}

/* Dekker's FastTwoSum: exact when a == 0 or |a| >= |b|. */
static inline odd fast_two_sum(double a, double b)
{
    odd r;
    double s = a + b;
    double e = b - (s - a);
    r.hi = s; r.lo = e;
    return r;
}

/* Exact product by fused multiply-add: a*b = p + e exactly. */
static inline odd two_prod(double a, double b)
{
    odd r;
    double p = a * b;
    double e = fma(a, b, -p);
    r.hi = p; r.lo = e;
    return r;
}

/* AccurateDWPlusDW (Joldes-Muller-Popescu 2017). */
static inline odd dd_add(odd x, odd y)
{
    odd s = two_sum(x.hi, y.hi);
    odd t = two_sum(x.lo, y.lo);
    double c = s.lo + t.hi;
    odd v = fast_two_sum(s.hi, c);
    double w = t.lo + v.lo;
    return fast_two_sum(v.hi, w);
}

/* DWTimesDW3 (Joldes-Muller-Popescu 2017). */
static inline odd dd_mul(odd x, odd y)
{
    odd c = two_prod(x.hi, y.hi);
    double t0 = x.lo * y.lo;
    double t1 = fma(x.hi, y.lo, t0);
    double c2 = fma(x.lo, y.hi, t1);
    double c3 = c.lo + c2;
    return fast_two_sum(c.hi, c3);
}

/* DWPlusFP (same paper): dd + binary64, relative error <= 2u^2. */
static inline odd dd_add_d(odd x, double y)
{
    odd s = two_sum(x.hi, y);
    double v = x.lo + s.lo;
    return fast_two_sum(s.hi, v);
}

/* DWTimesFP1 (Joldes-Muller-Popescu 2017): dd * binary64. */
static inline odd dd_mul_d(odd x, double y)
{
    odd c = two_prod(x.hi, y);
    double cl2 = x.lo * y;
    odd t = fast_two_sum(c.hi, cl2);
    double tl2 = t.lo + c.lo;
    return fast_two_sum(t.hi, tl2);
}

/* DWDivDW2 (Joldes-Muller-Popescu 2017): dd / dd, relative error
 * <= 15u^2 + 56u^3.  The quotient of the leading parts is corrected once by
 * the remainder x - y*t_h, whose leading part cancels exactly. */
static inline odd dd_div(odd x, odd y)
{
    double th = x.hi / y.hi;
    odd r = dd_mul_d(y, th);
    double pih = x.hi - r.hi;
    double dl = x.lo - r.lo;
    double d = pih + dl;
    double tl = d / y.hi;
    return fast_two_sum(th, tl);
}

/* Square root of a positive dd (Lefevre, Louvet, Muller, Picot, Rideau,
 * "Accurate calculation of Euclidean norms using double-word arithmetic",
 * ACM TOMS 2023: relative error <= 25/8 u^2): the binary64 root of the
 * leading part, corrected once with the exact remainder x.hi - s^2 (an fma)
 * plus the low part. */
static inline odd dd_sqrt(odd x)
{
    double sh = sqrt(x.hi);
    double r1 = fma(-sh, sh, x.hi);
    double r2 = x.lo + r1;
    double sl = r2 / (2.0 * sh);
    return fast_two_sum(sh, sl);
}

#endif

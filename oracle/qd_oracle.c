/*
 * qd_oracle.c -- CPU oracle for the quad-double (qd) Rgemm.
 *
 * TEST INFRASTRUCTURE ONLY (like dd_oracle.c): the slow, obviously-correct
 * reference the GPU library is checked against; it shares no code with the
 * GPU library.
 *
 * Number format (MPLAPACK 2.0.1 manual, section "Supported Floating point
 * formats"): a quad-double is the unevaluated sum x0 + x1 + x2 + x3 of four
 * binary64 numbers (QD library), about 64 decimal digits; Table "rlamch_qd"
 * gives its epsilon 2^-209.  A qd matrix is four column-major binary64
 * planes (x0, x1, x2, x3) with one leading dimension.
 *
 * What it computes: Rgemm on qd values, C <- alpha op(A) op(B) + beta C
 * (the DGEMM calling convention of section "How to use reference MPBLAS"),
 * with every entry the exact value rounded to a qd: the exact result V is
 * formed in a fixed-point accumulator wide enough for every binary64 product
 * that occurs, then x0 = RN(V), x1 = RN(V - x0), x2 = RN(V - x0 - x1),
 * x3 = RN(V - x0 - x1 - x2) (round to nearest, ties to even).  Each term of
 * alpha*a*b is a product of three binary64 numbers, split exactly into four
 * binary64 numbers by two levels of the fma product; beta*c into two.  So the
 * result does not depend on any choice of qd add / multiply algorithm; the GPU
 * kernels, which round as they go, are compared with it normwise.
 *
 * Argument checks and quick returns are BLAS DGEMM's (return value 0 or the
 * position of the first bad argument; nothing written when non-zero).
 * Supported range: every binary64 that occurs (inputs and the parts of their
 * products) has its exponent in [-1150, +1150); outside it the entry is NaN.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#define QACC_DIGITS 80                 /* 32-bit digits */
#define QACC_BASE (-1280)              /* weight of bit 0 of digit 0 */

typedef struct {
    int64_t d[QACC_DIGITS];            /* value = sum d[i] 2^(32 i + QACC_BASE) */
    int bad;                           /* a term fell outside the range */
    int64_t adds;
} qacc;

static void qacc_zero(qacc *a) { memset(a, 0, sizeof(*a)); }

/* carry-propagate so that 0 <= d[i] < 2^32 for every digit but the last */
static void qacc_norm(qacc *a)
{
    int i;
    for (i = 0; i < QACC_DIGITS - 1; ++i) {
        int64_t c = a->d[i] >> 32;     /* arithmetic shift: floor division */
        a->d[i] -= c * ((int64_t)1 << 32);
        a->d[i + 1] += c;
    }
    a->adds = 0;
}

static void qacc_add(qacc *a, double x)
{
    int e, pos, idx, sh;
    double fr;
    int64_t m;
    unsigned __int128 v;
    int neg = x < 0.0;
    if (x == 0.0) return;
    if (!isfinite(x)) { a->bad = 1; return; }
    fr = frexp(x, &e);                 /* x = fr 2^e, 0.5 <= |fr| < 1 */
    m = (int64_t)ldexp(fabs(fr), 53);  /* exact 53-bit integer */
    pos = e - 53 - QACC_BASE;          /* weight of m's bit 0 */
    if (pos < 0 || pos / 32 + 2 >= QACC_DIGITS) { a->bad = 1; return; }
    idx = pos / 32;
    sh = pos % 32;
    v = (unsigned __int128)m << sh;    /* < 2^85: three digits */
    if (neg) {
        a->d[idx] -= (int64_t)(v & 0xffffffffu);
        a->d[idx + 1] -= (int64_t)((v >> 32) & 0xffffffffu);
        a->d[idx + 2] -= (int64_t)(v >> 64);
    } else {
        a->d[idx] += (int64_t)(v & 0xffffffffu);
        a->d[idx + 1] += (int64_t)((v >> 32) & 0xffffffffu);
        a->d[idx + 2] += (int64_t)(v >> 64);
    }
    if (++a->adds >= ((int64_t)1 << 28)) qacc_norm(a);
}

/* exact two-term split of a product: a*b = p + e */
static void tp(double a, double b, double *p, double *e)
{
    *p = a * b;
    *e = fma(a, b, -*p);
}

/* a*b*c exactly as the sum of four binary64 numbers */
static void qacc_add3(qacc *acc, double a, double b, double c)
{
    double p1, e1, p2, e2, p3, e3;
    tp(a, b, &p1, &e1);
    tp(p1, c, &p2, &e2);
    tp(e1, c, &p3, &e3);
    qacc_add(acc, p2);
    qacc_add(acc, e2);
    qacc_add(acc, p3);
    qacc_add(acc, e3);
}

static void qacc_add2(qacc *acc, double a, double b)
{
    double p, e;
    tp(a, b, &p, &e);
    qacc_add(acc, p);
    qacc_add(acc, e);
}

/* nearest binary64 of the accumulated value (ties to even); the accumulator
 * must be normalised.  The value is not changed. */
static double qacc_round(const qacc *a)
{
    int64_t t[QACC_DIGITS];
    int i, h, neg, nb, shift, sticky = 0;
    unsigned __int128 N, mant, rem, half;
    memcpy(t, a->d, sizeof(t));
    neg = t[QACC_DIGITS - 1] < 0;
    if (neg) {                          /* two's complement negate, then renormalise */
        for (i = 0; i < QACC_DIGITS; ++i) t[i] = -t[i];
        for (i = 0; i < QACC_DIGITS - 1; ++i) {
            int64_t c = t[i] >> 32;
            t[i] -= c * ((int64_t)1 << 32);
            t[i + 1] += c;
        }
    }
    for (h = QACC_DIGITS - 1; h >= 0 && t[h] == 0; --h) {}
    if (h < 0) return 0.0;
    /* the top three digits (96 bits) and a sticky bit for the rest */
    N = 0;
    for (i = h; i >= h - 2; --i) N = (N << 32) | (unsigned __int128)(i >= 0 ? (uint64_t)t[i] : 0);
    for (i = h - 3; i >= 0; --i) if (t[i]) { sticky = 1; break; }
    nb = 0;
    for (rem = N; rem; rem >>= 1) ++nb;
    shift = nb - 53;                    /* >= 11: the top digit is non-zero */
    mant = N >> shift;
    rem = N & (((unsigned __int128)1 << shift) - 1);
    half = (unsigned __int128)1 << (shift - 1);
    if (rem > half || (rem == half && (sticky || (mant & 1)))) mant += 1;
    {
        double r = ldexp((double)(uint64_t)mant, shift + 32 * (h - 2) + QACC_BASE);
        return neg ? -r : r;
    }
}

static void qacc_to_qd(qacc *a, double q[4])
{
    int r;
    qacc_norm(a);
    for (r = 0; r < 4; ++r) {
        q[r] = qacc_round(a);
        qacc_add(a, -q[r]);
        qacc_norm(a);
    }
}

static int q_lsame(const char *s, char ref)
{
    char c;
    if (s == NULL) return 0;
    c = s[0];
    if (c >= 'a' && c <= 'z') c = (char)(c - 'a' + 'A');
    return c == ref;
}

static int q_zero(const double *x) { return x[0] == 0 && x[1] == 0 && x[2] == 0 && x[3] == 0; }
static int q_one(const double *x) { return x[0] == 1 && x[1] == 0 && x[2] == 0 && x[3] == 0; }

/* exported for the tests: round sum_i terms[i] (binary64) to a qd */
void oracle_qd_round_sum(int64_t count, const double *terms, double *q)
{
    qacc a;
    int64_t i;
    qacc_zero(&a);
    for (i = 0; i < count; ++i) qacc_add(&a, terms[i]);
    qacc_to_qd(&a, q);
    if (a.bad) q[0] = q[1] = q[2] = q[3] = NAN;
}

int oracle_Qgemm(const char *transa, const char *transb, int64_t m, int64_t n, int64_t k,
                 const double *alpha, const double *const *A, int64_t lda,
                 const double *const *B, int64_t ldb, const double *beta,
                 double *const *C, int64_t ldc)
{
    int nota = q_lsame(transa, 'N'), notb = q_lsame(transb, 'N');
    int64_t nrowa = nota ? m : k, nrowb = notb ? k : n, j;
    if (!nota && !q_lsame(transa, 'T') && !q_lsame(transa, 'C')) return 1;
    if (!notb && !q_lsame(transb, 'T') && !q_lsame(transb, 'C')) return 2;
    if (m < 0) return 3;
    if (n < 0) return 4;
    if (k < 0) return 5;
    if (lda < (nrowa > 1 ? nrowa : 1)) return 8;
    if (ldb < (nrowb > 1 ? nrowb : 1)) return 10;
    if (ldc < (m > 1 ? m : 1)) return 13;
    if (m == 0 || n == 0 || ((q_zero(alpha) || k == 0) && q_one(beta))) return 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (j = 0; j < n; ++j) {
        int64_t i, l;
        int r, p, q;
        qacc acc;
        for (i = 0; i < m; ++i) {
            const int64_t o = i + j * ldc;
            double out[4];
            qacc_zero(&acc);
            if (!q_zero(alpha) && k > 0) {
                for (l = 0; l < k; ++l) {
                    const int64_t ia = nota ? (i + l * lda) : (l + i * lda);
                    const int64_t ib = notb ? (l + j * ldb) : (j + l * ldb);
                    for (r = 0; r < 4; ++r) {
                        if (alpha[r] == 0.0) continue;
                        for (p = 0; p < 4; ++p)
                            for (q = 0; q < 4; ++q)
                                qacc_add3(&acc, alpha[r], A[p][ia], B[q][ib]);
                    }
                }
            }
            if (!q_zero(beta))
                for (r = 0; r < 4; ++r)
                    for (p = 0; p < 4; ++p) qacc_add2(&acc, beta[r], C[p][o]);
            qacc_to_qd(&acc, out);
            if (acc.bad) out[0] = out[1] = out[2] = out[3] = NAN;
            for (r = 0; r < 4; ++r) C[r][o] = out[r];
        }
    }
    return 0;
}

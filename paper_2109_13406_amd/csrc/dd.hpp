// dd.hpp -- double-double arithmetic for gfx950 device code.
//
// A dd value is the unevaluated sum hi + lo of two binary64 numbers (MPLAPACK
// manual, "Supported Floating point formats": dd_real, Knuth's and Dekker's
// error-free transformations).  All routines here are branch-free binary64
// sequences; FMA is always written explicitly and the library is compiled with
// -ffp-contract=off, so the compiler never fuses a multiply into an add.
//
//   two_sum       Knuth's TwoSum, 6 ops, exact for any a, b.
//   fast_two_sum  Dekker's FastTwoSum, 3 ops, exact when |a| >= |b| or a = 0.
//   two_prod      exact product via one v_fma_f64.
//   dd_add        AccurateDWPlusDW  (Joldes-Muller-Popescu 2017), rel. err. <= 3u^2.
//   dd_mul        DWTimesDW3        (same paper), rel. err. <= 4u^2.
//   dd_add_d      DWPlusFP          (same paper), rel. err. <= 2u^2.
//   madd_lean     acc += a*b with deferred renormalisation (10 ops, see below).
#pragma once
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace mpdd {

struct ddv {
  double hi, lo;
};

__device__ __forceinline__ ddv two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

__device__ __forceinline__ ddv fast_two_sum(double a, double b) {
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}

__device__ __forceinline__ ddv two_prod(double a, double b) {
  double p = a * b;
  double e = __builtin_fma(a, b, -p);
  return {p, e};
}

__device__ __forceinline__ ddv dd_add(ddv x, ddv y) {
  ddv s = two_sum(x.hi, y.hi);
  ddv t = two_sum(x.lo, y.lo);
  double c = s.lo + t.hi;
  ddv v = fast_two_sum(s.hi, c);
  double w = t.lo + v.lo;
  return fast_two_sum(v.hi, w);
}

__device__ __forceinline__ ddv dd_mul(ddv x, ddv y) {
  ddv c = two_prod(x.hi, y.hi);
  double t0 = x.lo * y.lo;
  double t1 = __builtin_fma(x.hi, y.lo, t0);
  double c2 = __builtin_fma(x.lo, y.hi, t1);
  double c3 = c.lo + c2;
  return fast_two_sum(c.hi, c3);
}

__device__ __forceinline__ ddv dd_add_d(ddv x, double y) {
  ddv s = two_sum(x.hi, y);
  double v = x.lo + s.lo;
  return fast_two_sum(s.hi, v);
}

// Accurate multiply-accumulate: acc <- dd_add(acc, dd_mul(a, b)); the same
// two published steps the reference evaluation uses (29 binary64 ops).
__device__ __forceinline__ void madd_accurate(double& sh, double& sl, double ah, double al,
                                              double bh, double bl) {
  ddv r = dd_add({sh, sl}, dd_mul({ah, al}, {bh, bl}));
  sh = r.hi;
  sl = r.lo;
}

// Lean multiply-accumulate (10 binary64 ops).  sh holds the running binary64
// sum of the leading products p = fl(ah*bh); every rounding error made on the
// way -- the product error ah*bh - p and the TwoSum error of sh + p -- and the
// cross terms ah*bl + al*bh are accumulated in sl.  al*bl (below u^2 |ab|) is
// dropped.  The pair is renormalised with two_sum once per staged k-tile, so
// |sl| stays near u |sh|; sh + sl carries ~106 bits.
//
// In TwoSum(sh, p) every operation after s = fl(sh + p) is exact, and its
// error is (sh - (s - bb)) + (p - bb) with bb = s - sh.  The product error and
// the second term together are ah*bh - bb exactly, which one fma evaluates
// with a single rounding; so the two error terms cost four ops after s (bb,
// s - bb, sh - (s - bb), the fma) instead of six, with the same O(u^2) error
// per term as adding the exact errors one by one.
__device__ __forceinline__ void madd_lean(double& sh, double& sl, double ah, double al,
                                          double bh, double bl) {
  double p = ah * bh;
  double s = sh + p;
  double bb = s - sh;
  double t2 = sh - (s - bb);
  double u = __builtin_fma(ah, bh, -bb);      // (p - bb) + (ah*bh - p), rounded once
  double t = __builtin_fma(ah, bl, sl);
  t = __builtin_fma(al, bh, t);
  sl = t + (t2 + u);
  sh = s;
}

// Lean multiply-accumulate without the cross terms (8 binary64 ops): the
// leading product and its rounding errors only; ah*bl + al*bh is accumulated
// elsewhere (on the matrix cores) and added to sl once per tile.
__device__ __forceinline__ void madd_lean_hi(double& sh, double& sl, double ah, double bh) {
  double p = ah * bh;
  double s = sh + p;
  double bb = s - sh;
  double t2 = sh - (s - bb);
  double u = __builtin_fma(ah, bh, -bb);      // (p - bb) + (ah*bh - p), rounded once
  sl = sl + (t2 + u);
  sh = s;
}

__device__ __forceinline__ void renorm(double& sh, double& sl) {
  ddv r = two_sum(sh, sl);
  sh = r.hi;
  sl = r.lo;
}

}  // namespace mpdd

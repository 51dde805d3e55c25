// dd_ext.hpp -- dd division and square root for gfx950 device code (used by
// the Cholesky kernels; the product kernels need only dd.hpp).
//
//   dd_mul_d  DWTimesFP1 (Joldes-Muller-Popescu 2017), dd * binary64.
//   dd_div    DWDivDW2 (same paper), relative error <= 15u^2 + 56u^3.
//   dd_sqrt   one remainder correction of the binary64 root (Lefevre, Louvet,
//             Muller, Picot, Rideau, ACM TOMS 2023), relative error <= 25/8 u^2.
#pragma once
#include "dd.hpp"

#pragma clang fp contract(off)

namespace mpdd {

__device__ __forceinline__ ddv dd_neg(ddv x) { return {-x.hi, -x.lo}; }

__device__ __forceinline__ ddv dd_mul_d(ddv x, double y) {
  ddv c = two_prod(x.hi, y);
  double cl2 = x.lo * y;
  ddv t = fast_two_sum(c.hi, cl2);
  double tl2 = t.lo + c.lo;
  return fast_two_sum(t.hi, tl2);
}

__device__ __forceinline__ ddv dd_div(ddv x, ddv y) {
  double th = x.hi / y.hi;
  ddv r = dd_mul_d(y, th);
  double pih = x.hi - r.hi;
  double dl = x.lo - r.lo;
  double d = pih + dl;
  double tl = d / y.hi;
  return fast_two_sum(th, tl);
}

__device__ __forceinline__ ddv dd_sqrt(ddv x) {
  double sh = __builtin_sqrt(x.hi);
  double r1 = __builtin_fma(-sh, sh, x.hi);
  double r2 = x.lo + r1;
  double sl = r2 / (2.0 * sh);
  return fast_two_sum(sh, sl);
}

}  // namespace mpdd

// qd.hpp -- quad-double accumulation on gfx950, shared by the qd Rgemm
// kernels (qd.hip) and the split-form qd combine (ozaki.hip).
//
// A quad-double is x0 + x1 + x2 + x3, four binary64 numbers.  The
// accumulator keeps one binary64 per level of magnitude 2^(-53 L) of the
// leading part; see qd.hip for the multiply-accumulate by levels.
#pragma once
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace mpdd {
namespace {

struct qacc {
  double s0, s1, s2, s3;
};

__device__ __forceinline__ void ts(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void tp(double a, double b, double& p, double& e) {
  p = a * b;
  e = __builtin_fma(a, b, -p);
}

// s2 += fl(a*b) by TwoSum, returning the level-3 residue: the TwoSum error
// (s2 - (s - bb)) + (p - bb) plus the product error a*b - p.  The last two add
// up to a*b - bb exactly, which one fma gives with a single rounding (an error
// of a level-3 size times 2^-53, like the plain additions of level 3).
__device__ __forceinline__ double ts_prod(double& s2, double a, double b) {
  const double p = a * b;
  const double s = s2 + p;
  const double bb = s - s2;
  const double t2 = s2 - (s - bb);
  const double u = __builtin_fma(a, b, -bb);
  s2 = s;
  return t2 + u;
}

// c += a * b by levels (see the file comment)
__device__ __forceinline__ void qd_madd(qacc& c, const double4& a, const double4& b) {
  double p00, e00, p01, e01, p10, e10;
  tp(a.x, b.x, p00, e00);
  tp(a.x, b.y, p01, e01);
  tp(a.y, b.x, p10, e10);
  double l3 = a.w * b.x;
  l3 = __builtin_fma(a.z, b.y, l3);
  l3 = __builtin_fma(a.y, b.z, l3);
  l3 = __builtin_fma(a.x, b.w, l3);
  l3 = __builtin_fma(a.y, b.w, l3);
  l3 = __builtin_fma(a.z, b.z, l3);
  l3 = __builtin_fma(a.w, b.y, l3);
  double t1, u1, u2, u3, u4, v;
  double w = 0.0;
  // level 0
  ts(c.s0, p00, c.s0, t1);
  // level 1
  ts(c.s1, t1, c.s1, u1);
  ts(c.s1, e00, c.s1, u2);
  ts(c.s1, p01, c.s1, u3);
  ts(c.s1, p10, c.s1, u4);
  // level 2
  ts(c.s2, u1, c.s2, v); w += v;
  ts(c.s2, u2, c.s2, v); w += v;
  ts(c.s2, u3, c.s2, v); w += v;
  ts(c.s2, u4, c.s2, v); w += v;
  ts(c.s2, e01, c.s2, v); w += v;
  ts(c.s2, e10, c.s2, v); w += v;
  // a0b2, a1b1, a2b0 with their product errors (level 3) folded in
  w += ts_prod(c.s2, a.x, b.z);
  w += ts_prod(c.s2, a.y, b.y);
  w += ts_prod(c.s2, a.z, b.x);
  // level 3
  c.s3 = c.s3 + (w + l3);
}

// two TwoSum sweeps: bottom-up (the sum gathers in s0), then top-down
__device__ __forceinline__ void qd_renorm(qacc& c) {
  ts(c.s2, c.s3, c.s2, c.s3);
  ts(c.s1, c.s2, c.s1, c.s2);
  ts(c.s0, c.s1, c.s0, c.s1);
  ts(c.s1, c.s2, c.s1, c.s2);
  ts(c.s2, c.s3, c.s2, c.s3);
}

// final normalisation to a qd with non-overlapping parts
__device__ __forceinline__ double4 qd_final(qacc c) {
  qd_renorm(c);
  qd_renorm(c);
  ts(c.s0, c.s1, c.s0, c.s1);
  ts(c.s1, c.s2, c.s1, c.s2);
  ts(c.s2, c.s3, c.s2, c.s3);
  return double4{c.s0, c.s1, c.s2, c.s3};
}

}  // namespace
}  // namespace mpdd

// complex.hip -- elementwise complex dd kernel of Cgemm.
//
// Cgemm (MPLAPACK manual, section "How to use reference MPBLAS", the Cgemm
// part: ZGEMM's calling convention on complex multiple-precision values)
// runs its four real products op(A)_{re,im} op(B)_{re,im} on the plain dd
// kernels into a product P = op(A) op(B) held as two dd planes pairs (or, for
// the three-product form, into R1, R2, R3 from which P is formed here); this
// kernel then forms C <- alpha P + beta C in complex dd arithmetic, or
// C <- beta C (alpha = 0 or k = 0).  dd_axpy_planes forms the operand sums of
// the three-product form.  A complex product is
//   (a + ib)(c + id) = (ac - bd) + i(ad + bc),
// each real product a dd multiply and each sum a dd add.
//
// HBM-bound: one pass over P (32 B per entry) and C (32 B read unless
// beta = 0, 32 B written).
#include "dd.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace mpdd {

namespace {

__device__ __forceinline__ ddv dd_neg(ddv x) { return {-x.hi, -x.lo}; }

__device__ __forceinline__ void cmul(ddv xr, ddv xi, ddv yr, ddv yi, ddv& zr, ddv& zi) {
  zr = dd_add(dd_mul(xr, yr), dd_neg(dd_mul(xi, yi)));
  zi = dd_add(dd_mul(xr, yi), dd_mul(xi, yr));
}

__global__ void __launch_bounds__(256) dd_cgemm_epilogue(CEpilogue p) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= p.m * p.n) return;
  const int64_t i = gid % p.m, j = gid / p.m;
  const int64_t ci = i + j * p.ldc;
  const ddv ar{p.alpha[0], p.alpha[1]}, ai{p.alpha[2], p.alpha[3]};
  const ddv br{p.beta[0], p.beta[1]}, bi{p.beta[2], p.beta[3]};
  ddv zr{0.0, 0.0}, zi{0.0, 0.0};
  if (p.use_p) {
    const int64_t pi = i + j * p.ldp;
    ddv pr{p.p_rh[pi], p.p_rl[pi]}, pim{p.p_ih[pi], p.p_il[pi]};
    if (p.three_m) {
      // R1 = pr, R2 = pim, R3 = q: P = (R1 - R2) + i (R3 - R1 - R2)
      const ddv r3{p.q_h[pi], p.q_l[pi]};
      const ddv s12 = dd_add(pr, pim);
      const ddv re = dd_add(pr, dd_neg(pim));
      pim = dd_add(r3, dd_neg(s12));
      pr = re;
    }
    cmul(ar, ai, pr, pim, zr, zi);
    if (!p.beta_zero) {
      ddv tr, ti;
      cmul(br, bi, ddv{p.c_rh[ci], p.c_rl[ci]}, ddv{p.c_ih[ci], p.c_il[ci]}, tr, ti);
      zr = dd_add(zr, tr);
      zi = dd_add(zi, ti);
    }
  } else if (!p.beta_zero) {
    cmul(br, bi, ddv{p.c_rh[ci], p.c_rl[ci]}, ddv{p.c_ih[ci], p.c_il[ci]}, zr, zi);
  }
  p.c_rh[ci] = zr.hi;
  p.c_rl[ci] = zr.lo;
  p.c_ih[ci] = zi.hi;
  p.c_il[ci] = zi.lo;
}

__global__ void __launch_bounds__(256)
dd_axpy_planes(const double* __restrict__ xh, const double* __restrict__ xl,
               const double* __restrict__ yh, const double* __restrict__ yl, int64_t ld, double s,
               int64_t rows, int64_t cols, double* __restrict__ oh, double* __restrict__ ol) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= rows * cols) return;
  const int64_t i = gid % rows, j = gid / rows;
  const int64_t o = i + j * ld;
  const ddv r = dd_add(ddv{xh[o], xl[o]}, ddv{s * yh[o], s * yl[o]});
  oh[gid] = r.hi;
  ol[gid] = r.lo;
}

}  // namespace

hipError_t launch_dd_axpy_planes(const double* x_hi, const double* x_lo, const double* y_hi,
                                 const double* y_lo, int64_t ld, double s, int64_t rows,
                                 int64_t cols, double* o_hi, double* o_lo, hipStream_t st) {
  const int64_t total = rows * cols;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(dd_axpy_planes, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     x_hi, x_lo, y_hi, y_lo, ld, s, rows, cols, o_hi, o_lo);
  return hipGetLastError();
}

hipError_t launch_cgemm_epilogue(const CEpilogue& p, hipStream_t st) {
  const int64_t total = p.m * p.n;
  hipLaunchKernelGGL(dd_cgemm_epilogue, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     p);
  return hipGetLastError();
}

}  // namespace mpdd

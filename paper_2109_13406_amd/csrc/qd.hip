// qd.hip -- quad-double Rgemm kernels for gfx950.
//
// A quad-double (MPLAPACK manual, section "Supported Floating point formats":
// qd_real of the QD library, about 64 digits, epsilon 2^-209 in Table
// "rlamch_qd") is x0 + x1 + x2 + x3, four binary64 numbers; a qd matrix is
// four column-major binary64 planes with one leading dimension.  Rgemm on qd
// values: C <- alpha op(A) op(B) + beta C.
//
// Multiply-accumulate by levels.  With |a_t|, |b_t| <= 2^(-53 t) |a_0|, |b_0|,
// the partial products a_p b_q and their fma errors fall into levels 0..3 of
// magnitude 2^(-53 L) |a0 b0|:
//   level 0: a0b0;  level 1: err(a0b0), a0b1, a1b0;
//   level 2: err(a0b1), err(a1b0), a0b2, a1b1, a2b0;
//   level 3: err(a0b2), err(a1b1), err(a2b0), a0b3 + a1b2 + a2b1 + a3b0
//            + a1b3 + a2b2 + a3b1 (fma chain).
// The accumulator keeps one binary64 per level.  Adding a level-L term uses
// TwoSum for L = 0, 1, 2, its rounding error going to level L+1; level-3 terms
// are added plainly (their errors are below 2^-212 relative).  What is dropped
// per term (the errors of the level-3 products and of their fma chain, and
// a2b3 + a3b2 + a3b3) is a few units of 2^-212 |ab|.  The four levels are
// renormalised (two TwoSum sweeps) once per staged k-tile, so that each level
// stays near 2^-53 of the one above.
//
// Tile: 32 x 32 outputs per workgroup of 256 threads, 2 x 2 outputs per thread
// (rows tm + 16 r, columns tn + 16 c), k staged QD_BK deep through LDS as
// double4 (x0..x3) entries.  About 110 binary64 operations per multiply-add,
// so the kernel is FP64-issue-bound like the dd kernels.
#include "dd.hpp"
#include "kernels.hpp"
#include "qd.hpp"

#pragma clang fp contract(off)

namespace mpdd {

namespace {

constexpr int QD_BM = 32, QD_BN = 32, QD_BK = 8;

__device__ __forceinline__ double4 qd_load(const QgemmParams& p, int which, int64_t idx) {
  const double* const* pl = which == 0 ? p.a : (which == 1 ? p.b : (const double* const*)p.c);
  return double4{pl[0][idx], pl[1][idx], pl[2][idx], pl[3][idx]};
}

// C = alpha * acc + beta * C (beta_zero: C not read), as qd products summed
// by levels and normalised
__device__ __forceinline__ double4 qd_epilogue(const QgemmParams& p, const double4& accq,
                                               int64_t ci) {
  qacc r{0.0, 0.0, 0.0, 0.0};
  const double4 al{p.alpha[0], p.alpha[1], p.alpha[2], p.alpha[3]};
  qd_madd(r, al, accq);
  if (!p.beta_zero) {
    const double4 be{p.beta[0], p.beta[1], p.beta[2], p.beta[3]};
    const double4 c0{p.c[0][ci], p.c[1][ci], p.c[2][ci], p.c[3][ci]};
    qd_renorm(r);
    qd_madd(r, be, c0);
  }
  return qd_final(r);
}

template <bool TA, bool TB>
__global__ void __launch_bounds__(256) qd_gemm_kernel(QgemmParams p) {
  __shared__ double4 As[QD_BK][QD_BM];
  __shared__ double4 Bs[QD_BK][QD_BN];
  const int tid = threadIdx.x;
  const int tm = tid % 16, tn = tid / 16;
  const int64_t i0 = (int64_t)blockIdx.x * QD_BM, j0 = (int64_t)blockIdx.y * QD_BN;

  qacc acc[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[r][c] = qacc{0.0, 0.0, 0.0, 0.0};

  // staging: thread -> (row-of-tile, k) for A and (col-of-tile, k) for B
  const int ar = TA ? tid / QD_BK : tid % QD_BM, ak = TA ? tid % QD_BK : tid / QD_BM;
  const int bc = TB ? tid % QD_BN : tid / QD_BK, bk = TB ? tid / QD_BN : tid % QD_BK;
  const int64_t gi = i0 + ar, gj = j0 + bc;
  for (int64_t l0 = 0; l0 < p.k; l0 += QD_BK) {
    {
      const int64_t l = l0 + ak;
      double4 v{0.0, 0.0, 0.0, 0.0};
      if (gi < p.m && l < p.k) v = qd_load(p, 0, TA ? (l + gi * p.lda) : (gi + l * p.lda));
      As[ak][ar] = v;
    }
    {
      const int64_t l = l0 + bk;
      double4 v{0.0, 0.0, 0.0, 0.0};
      if (gj < p.n && l < p.k) v = qd_load(p, 1, TB ? (gj + l * p.ldb) : (l + gj * p.ldb));
      Bs[bk][bc] = v;
    }
    __syncthreads();
#pragma unroll 2
    for (int kk = 0; kk < QD_BK; ++kk) {
      const double4 a0 = As[kk][tm], a1 = As[kk][tm + 16];
      const double4 b0 = Bs[kk][tn], b1 = Bs[kk][tn + 16];
      qd_madd(acc[0][0], a0, b0);
      qd_madd(acc[0][1], a0, b1);
      qd_madd(acc[1][0], a1, b0);
      qd_madd(acc[1][1], a1, b1);
    }
    // renormalise once per staged k-tile (QD_BK terms)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) qd_renorm(acc[r][c]);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int64_t i = i0 + tm + 16 * r;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int64_t j = j0 + tn + 16 * c;
      if (i >= p.m || j >= p.n) continue;
      const int64_t ci = i + j * p.ldc;
      const double4 v = qd_epilogue(p, qd_final(acc[r][c]), ci);
      p.c[0][ci] = v.x;
      p.c[1][ci] = v.y;
      p.c[2][ci] = v.z;
      p.c[3][ci] = v.w;
    }
  }
}

// C <- beta * C (alpha = 0 or k = 0); beta = 0 writes zeros without reading C
__global__ void __launch_bounds__(256) qd_scale_kernel(QgemmParams p) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= p.m * p.n) return;
  const int64_t i = gid % p.m, j = gid / p.m;
  const int64_t ci = i + j * p.ldc;
  double4 v{0.0, 0.0, 0.0, 0.0};
  if (!p.beta_zero) {
    qacc r{0.0, 0.0, 0.0, 0.0};
    const double4 be{p.beta[0], p.beta[1], p.beta[2], p.beta[3]};
    qd_madd(r, be, double4{p.c[0][ci], p.c[1][ci], p.c[2][ci], p.c[3][ci]});
    v = qd_final(r);
  }
  p.c[0][ci] = v.x;
  p.c[1][ci] = v.y;
  p.c[2][ci] = v.z;
  p.c[3][ci] = v.w;
}

}  // namespace

hipError_t launch_qgemm(const QgemmParams& p, bool ta, bool tb, hipStream_t st) {
  if (p.scale_only) {
    const int64_t total = p.m * p.n;
    hipLaunchKernelGGL(qd_scale_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       p);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((p.m + QD_BM - 1) / QD_BM), (unsigned)((p.n + QD_BN - 1) / QD_BN));
  auto kern = !ta ? (!tb ? qd_gemm_kernel<false, false> : qd_gemm_kernel<false, true>)
                  : (!tb ? qd_gemm_kernel<true, false> : qd_gemm_kernel<true, true>);
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, p);
  return hipGetLastError();
}

}  // namespace mpdd

// potrf.hip -- diagonal-block kernel of the blocked dd Cholesky (Rpotrf).
//
// Rpotrf (MPLAPACK: LAPACK's DPOTRF on multiple-precision values) factors a
// symmetric positive definite A as L L^T (uplo 'L') or U^T U (uplo 'U').
// The blocked driver (mpdd.cpp) runs the O(n^3) work on the plain dd product
// kernels and calls this kernel once per diagonal block of order jb <= 64:
// it reads the updated block from the driver's panel copy (s, ld lds) and
// writes the factor to A (ld lda).  It works in the "lower view" L(i, l) of
// the block (L(i, l) = A(i, l) for 'L', A(l, i) for 'U'):
//
//   1. right-looking Cholesky of the block in place, column by column:
//      pivot d = L(c,c); d <= 0 or NaN -> info = offset + c+1 and stop (d
//      stays in place); L(c,c) = sqrt(d); L(i,c) /= L(c,c); then the
//      trailing lower triangle L(i,l) -= L(i,c) L(l,c).  The info word is
//      shared by the blocks of one factorisation: a block that finds it set
//      returns at once, so only the first failure is recorded;
//   2. the inverse W = L^-1 (lower triangular, ld jb, zeros above the
//      diagonal), row by row: W(i,i) = 1 / L(i,i) and, for t < i,
//      W(i,t) = -(sum_{t<=l<i} L(i,l) W(l,t)) / L(i,i).  The panel solve of
//      the driver is then a plain dd product with W, on the product kernels.
//
// One workgroup of 512 threads.  The block's lower triangle and W live in LDS
// (packed by rows, 4 x 16.6 KB), so each of the O(jb) dependent steps costs
// LDS latency, not a global-memory round trip; the block is read once and
// written once.  All arithmetic is the
// accurate dd add / multiply of dd.hpp and the division / square root of
// dd_ext.hpp.
#include "dd_ext.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace mpdd {

namespace {

constexpr int POTF2_MAX = 64;       // largest block order
constexpr int POTF2_THREADS = 512;
constexpr int POTF2_LANES = 8;      // lanes per column of W in step 2
constexpr int POTF2_PACK = POTF2_MAX * (POTF2_MAX + 1) / 2;

__device__ __forceinline__ int64_t lv(int upper, int64_t i, int64_t l, int64_t lda) {
  return upper ? (l + i * lda) : (i + l * lda);
}

// packed lower triangle, row by row: (i, l), l <= i
__device__ __forceinline__ int pk(int i, int l) { return i * (i + 1) / 2 + l; }

__global__ void __launch_bounds__(POTF2_THREADS)
dd_potf2_block(const double* __restrict__ s_hi, const double* __restrict__ s_lo, int64_t lds,
               double* __restrict__ a_hi, double* __restrict__ a_lo, int64_t lda, int jb,
               int upper, double* __restrict__ w_hi, double* __restrict__ w_lo,
               long long* __restrict__ info, long long offset) {
  __shared__ double lh[POTF2_PACK], ll[POTF2_PACK], wh[POTF2_PACK], wl[POTF2_PACK];
  __shared__ int s_fail;
  // an earlier block of this factorisation failed: leave this one alone
  if (*info != 0) return;
  const int tid = threadIdx.x;
  if (tid == 0) s_fail = 0;
  for (int t = tid; t < jb * jb; t += POTF2_THREADS) {
    const int i = t % jb, l = t / jb;
    if (i < l) continue;
    const int64_t o = lv(upper, i, l, lds);
    lh[pk(i, l)] = s_hi[o];
    ll[pk(i, l)] = s_lo[o];
  }
  __syncthreads();

  // 1. right-looking factorisation in LDS
  for (int c = 0; c < jb; ++c) {
    if (tid == 0) {
      const ddv d{lh[pk(c, c)], ll[pk(c, c)]};
      if (!(d.hi > 0.0)) {
        s_fail = c + 1;
      } else {
        const ddv p = dd_sqrt(d);
        lh[pk(c, c)] = p.hi;
        ll[pk(c, c)] = p.lo;
      }
    }
    __syncthreads();
    if (s_fail) break;
    const ddv piv{lh[pk(c, c)], ll[pk(c, c)]};
    for (int i = c + 1 + tid; i < jb; i += POTF2_THREADS) {
      const ddv q = dd_div(ddv{lh[pk(i, c)], ll[pk(i, c)]}, piv);
      lh[pk(i, c)] = q.hi;
      ll[pk(i, c)] = q.lo;
    }
    __syncthreads();
    const int m = jb - c - 1;
    for (int t = tid; t < m * m; t += POTF2_THREADS) {
      const int i = c + 1 + t % m, l = c + 1 + t / m;
      if (i < l) continue;
      const ddv p = dd_mul(ddv{lh[pk(i, c)], ll[pk(i, c)]}, ddv{lh[pk(l, c)], ll[pk(l, c)]});
      const ddv r = dd_add(ddv{lh[pk(i, l)], ll[pk(i, l)]}, dd_neg(p));
      lh[pk(i, l)] = r.hi;
      ll[pk(i, l)] = r.lo;
    }
    __syncthreads();
  }
  const int fail = s_fail;

  // 2. W = L^-1, row by row (8 lanes per column, fixed-order butterfly)
  if (!fail) {
    const int col = tid / POTF2_LANES, q = tid % POTF2_LANES;
    for (int i = 0; i < jb; ++i) {
      if (col < i) {
        ddv s{0.0, 0.0};
        for (int l = col + q; l < i; l += POTF2_LANES)
          s = dd_add(s, dd_mul(ddv{lh[pk(i, l)], ll[pk(i, l)]}, ddv{wh[pk(l, col)], wl[pk(l, col)]}));
#pragma unroll
        for (int x = 1; x < POTF2_LANES; x <<= 1) {
          const ddv o{__shfl_xor(s.hi, x), __shfl_xor(s.lo, x)};
          s = (q & x) ? dd_add(o, s) : dd_add(s, o);
        }
        if (q == 0) {
          const ddv r = dd_neg(dd_div(s, ddv{lh[pk(i, i)], ll[pk(i, i)]}));
          wh[pk(i, col)] = r.hi;
          wl[pk(i, col)] = r.lo;
        }
      } else if (col == i && q == 0) {
        const ddv r = dd_div(ddv{1.0, 0.0}, ddv{lh[pk(i, i)], ll[pk(i, i)]});
        wh[pk(i, i)] = r.hi;
        wl[pk(i, i)] = r.lo;
      }
      __syncthreads();
    }
  }

  // write back the (partial, on failure) factor, and W with zeros above its diagonal
  for (int t = tid; t < jb * jb; t += POTF2_THREADS) {
    const int i = t % jb, l = t / jb;
    if (i < l) {
      if (!fail) {
        w_hi[t] = 0.0;
        w_lo[t] = 0.0;
      }
      continue;
    }
    const int64_t o = lv(upper, i, l, lda);
    a_hi[o] = lh[pk(i, l)];
    a_lo[o] = ll[pk(i, l)];
    if (!fail) {
      w_hi[t] = wh[pk(i, l)];
      w_lo[t] = wl[pk(i, l)];
    }
  }
  if (tid == 0 && fail) *info = offset + fail;
}

}  // namespace

hipError_t launch_potf2_block(const double* s_hi, const double* s_lo, int64_t lds, double* a_hi,
                              double* a_lo, int64_t lda, int jb, int upper, double* w_hi,
                              double* w_lo, long long* info, long long offset, hipStream_t st) {
  if (jb < 1 || jb > POTF2_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dd_potf2_block, dim3(1), dim3(POTF2_THREADS), 0, st, s_hi, s_lo, lds, a_hi,
                     a_lo, lda, jb, upper, w_hi, w_lo, info, offset);
  return hipGetLastError();
}

}  // namespace mpdd

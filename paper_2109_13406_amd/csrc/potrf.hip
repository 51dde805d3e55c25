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
//   right-looking Cholesky of the block in place, column by column, with the
//   inverse W = L^-1 built in the same sweep (W starts as the identity; the
//   forward elimination of L W = I proceeds in the column order of the
//   factorisation).  For column c:
//     A. pivot d = L(c,c); d <= 0 or NaN -> info = offset + c+1 and stop (d
//        stays in place); p = sqrt(d) (every thread that needs it computes the
//        same value itself); L(c,c) = p; L(i,c) /= p for i > c; row c of W,
//        final apart from this step, is divided by p (W(c,c) = 1/p);
//     B. trailing lower triangle L(i,l) -= L(i,c) L(l,c) for c < l <= i, and
//        W(i,t) -= L(i,c) W(c,t) for i > c, t <= c.
//   One barrier after each phase.  The info word is shared by the blocks of
//   one factorisation: a block that finds it set returns at once, so only the
//   first failure is recorded.  The panel solve of the driver is then a plain
//   dd product with W, on the product kernels.
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
  // This workgroup is the critical path of the factorisation and shares its
  // CU with the workgroups of the bulk update running beside it: raise its
  // waves' issue priority so that their dependent chains are not starved.
  __builtin_amdgcn_s_setprio(3);
  // an earlier block of this factorisation failed: leave this one alone
  if (*info != 0) return;
  const int tid = threadIdx.x;
  for (int t = tid; t < jb * jb; t += POTF2_THREADS) {
    const int i = t % jb, l = t / jb;
    if (i < l) continue;
    const int64_t o = lv(upper, i, l, lds);
    lh[pk(i, l)] = s_hi[o];
    ll[pk(i, l)] = s_lo[o];
    wh[pk(i, l)] = (i == l) ? 1.0 : 0.0;
    wl[pk(i, l)] = 0.0;
  }
  __syncthreads();

  int fail = 0;
  for (int c = 0; c < jb; ++c) {
    const int m = jb - c - 1;
    // A. pivot, column c of L, row c of W (m + c + 1 = jb <= 64 items: wave 0).
    //    L(c,c) itself is overwritten only in phase B, when no thread reads it.
    const ddv d{lh[pk(c, c)], ll[pk(c, c)]};
    if (!(d.hi > 0.0)) {            // the same decision in every thread
      fail = c + 1;
      break;
    }
    ddv piv{0.0, 0.0};
    if (tid < m + c + 1) {
      piv = dd_sqrt(d);
      if (tid < m) {
        const int i = c + 1 + tid;
        const ddv q = dd_div(ddv{lh[pk(i, c)], ll[pk(i, c)]}, piv);
        lh[pk(i, c)] = q.hi;
        ll[pk(i, c)] = q.lo;
      } else {
        const int t = tid - m;      // 0 .. c
        const ddv q = dd_div(ddv{wh[pk(c, t)], wl[pk(c, t)]}, piv);
        wh[pk(c, t)] = q.hi;
        wl[pk(c, t)] = q.lo;
      }
    }
    __syncthreads();
    if (tid == 0) {
      lh[pk(c, c)] = piv.hi;
      ll[pk(c, c)] = piv.lo;
    }
    // B. trailing triangle of L (m * m slots, upper half skipped) and rows
    //    c+1 .. jb-1 of W in columns 0 .. c
    const int nl = m * m, nw = m * (c + 1);
    for (int q = tid; q < nl + nw; q += POTF2_THREADS) {
      if (q < nl) {
        const int i = c + 1 + q % m, l = c + 1 + q / m;
        if (i < l) continue;
        const ddv p = dd_mul(ddv{lh[pk(i, c)], ll[pk(i, c)]}, ddv{lh[pk(l, c)], ll[pk(l, c)]});
        const ddv r = dd_add(ddv{lh[pk(i, l)], ll[pk(i, l)]}, dd_neg(p));
        lh[pk(i, l)] = r.hi;
        ll[pk(i, l)] = r.lo;
      } else {
        const int r0 = q - nl;
        const int i = c + 1 + r0 % m, t = r0 / m;
        const ddv p = dd_mul(ddv{lh[pk(i, c)], ll[pk(i, c)]}, ddv{wh[pk(c, t)], wl[pk(c, t)]});
        const ddv r = dd_add(ddv{wh[pk(i, t)], wl[pk(i, t)]}, dd_neg(p));
        wh[pk(i, t)] = r.hi;
        wl[pk(i, t)] = r.lo;
      }
    }
    __syncthreads();
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

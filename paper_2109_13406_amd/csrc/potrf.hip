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
//   factorisation).  Finishing column c means: pivot d = L(c,c) (after the
//   updates of columns < c); d <= 0 or NaN -> info = offset + c+1 and stop
//   (d stays in place); p = sqrt(d); L(c,c) = p; L(i,c) *= 1/p for i > c
//   and row c of W is multiplied by 1/p (W(c,c) = 1/p), with 1/p the dd
//   reciprocal, formed once.  Column c then updates the
//   trailing triangle, L(i,l) -= L(i,c) L(l,c) for c < l <= i, and W(i,t) -=
//   L(i,c) W(c,t) for i > c, t <= c.
//
//   Look-ahead, one barrier per column: while waves 1-15 apply column c to the
//   trailing entries outside column c+1 and row c+1 of W, wave 0 applies it to
//   column c+1 and row c+1 of W (jb entries, one per lane), takes the updated
//   pivot from lane 0 by a cross-lane broadcast and finishes column c+1.
//   Every entry receives the same operations in the same order as in the
//   plain column sweep.
//
// One workgroup of 1024 threads.  The block's lower triangle and W live in LDS
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
constexpr int POTF2_THREADS = 1024;
constexpr int POTF2_PACK = POTF2_MAX * (POTF2_MAX + 1) / 2;

__device__ __forceinline__ int64_t lv(int upper, int64_t i, int64_t l, int64_t lda) {
  return upper ? (l + i * lda) : (i + l * lda);
}

// packed lower triangle, row by row: (i, l), l <= i
__device__ __forceinline__ int pk(int i, int l) { return i * (i + 1) / 2 + l; }

// x of the wave's first active lane, to every lane (two scalar reads; no
// LDS round trip)
__device__ __forceinline__ double first_lane(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__global__ void __launch_bounds__(POTF2_THREADS)
dd_potf2_block(const double* __restrict__ s_hi, const double* __restrict__ s_lo, int64_t lds,
               double* __restrict__ a_hi, double* __restrict__ a_lo, int64_t lda, int jb,
               int upper, double* __restrict__ w_hi, double* __restrict__ w_lo,
               long long* __restrict__ info, long long offset) {
  __shared__ double lh[POTF2_PACK], ll[POTF2_PACK], wh[POTF2_PACK], wl[POTF2_PACK];
  // row r of packed index q = r (r + 1) / 2 + x (x <= r) of a triangle, for
  // the trailing updates (filled once; replaces a square root per entry)
  __shared__ unsigned char tri_row[POTF2_PACK];
  // This workgroup is the critical path of the factorisation and shares its
  // CU with the workgroups of the bulk update running beside it: raise its
  // waves' issue priority so that their dependent chains are not starved,
  // wave 0 (which finishes each next column) above the others.
  if (threadIdx.x < 64)
    __builtin_amdgcn_s_setprio(3);
  else
    __builtin_amdgcn_s_setprio(2);
  // an earlier block of this factorisation failed: leave this one alone
  if (*info != 0) return;
  const int tid = threadIdx.x;
  for (int q = tid; q < POTF2_PACK; q += POTF2_THREADS) {
    int r = (int)((__builtin_sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
    if ((r + 1) * (r + 2) / 2 <= q) ++r;
    if (r * (r + 1) / 2 > q) --r;
    tri_row[q] = (unsigned char)r;
  }
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

  const int lane = tid & 63;
  // finish column 0 (wave 0); a failing pivot is left in place.  The column
  // is scaled by the dd reciprocal of the pivot, which every lane forms (one
  // division on the dependent path instead of two divergent ones)
  if (tid < 64) {
    const ddv d{lh[0], ll[0]};
    if (d.hi > 0.0) {
      const ddv piv = dd_sqrt(d);
      const ddv inv = dd_div(ddv{1.0, 0.0}, piv);
      if (lane >= 1 && lane < jb) {
        const ddv q = dd_mul(ddv{lh[pk(lane, 0)], ll[pk(lane, 0)]}, inv);
        lh[pk(lane, 0)] = q.hi;
        ll[pk(lane, 0)] = q.lo;
      } else if (lane == 0) {
        wh[0] = inv.hi;
        wl[0] = inv.lo;
        lh[0] = piv.hi;
        ll[0] = piv.lo;
      }
    }
  }
  __syncthreads();

  int fail = 0;
  for (int c = 0; c < jb; ++c) {
    // column c is finished unless its pivot failed (nobody writes L(c,c)
    // during this step, so every thread takes the same decision)
    if (!(lh[pk(c, c)] > 0.0)) {
      fail = c + 1;
      break;
    }
    const int m = jb - c - 1;           // rows below the pivot
    if (tid < 64) {
      if (m > 0) {
        // column c+1 (lanes 0 .. m-1: rows c+1 .. jb-1; lane 0 holds the
        // pivot) and row c+1 of W (lanes m .. m+c: columns 0 .. c)
        const ddv lc1{lh[pk(c + 1, c)], ll[pk(c + 1, c)]};      // L(c+1, c)
        int o = 0;
        bool in_w = false, active = lane < m + c + 1;
        ddv z{0.0, 0.0};
        if (lane < m) {
          const int i = c + 1 + lane;
          o = pk(i, c + 1);
          z = dd_add(ddv{lh[o], ll[o]}, dd_neg(dd_mul(ddv{lh[pk(i, c)], ll[pk(i, c)]}, lc1)));
        } else if (active) {
          const int t = lane - m;
          o = pk(c + 1, t);
          in_w = true;
          z = dd_add(ddv{wh[o], wl[o]}, dd_neg(dd_mul(lc1, ddv{wh[pk(c, t)], wl[pk(c, t)]})));
        }
        // the updated pivot, from lane 0 (every lane of the wave is active
        // here) to the whole wave
        const ddv d{first_lane(z.hi), first_lane(z.lo)};
        if (d.hi > 0.0) {
          const ddv piv = dd_sqrt(d);
          const ddv inv = dd_div(ddv{1.0, 0.0}, piv);     // W(c+1,c+1) = 1 / p
          if (lane == 0) {
            wh[pk(c + 1, c + 1)] = inv.hi;
            wl[pk(c + 1, c + 1)] = inv.lo;
            z = piv;
          } else if (active) {
            z = dd_mul(z, inv);
          }
        }
        if (active) {
          if (in_w) {
            wh[o] = z.hi;
            wl[o] = z.lo;
          } else {
            lh[o] = z.hi;
            ll[o] = z.lo;
          }
        }
      }
    } else if (m > 1) {
      // the rest of column c's update: L(i,l), c+2 <= l <= i (packed row by
      // row), then W(i,t), i >= c+2, t <= c
      const int m2 = m - 1;
      const int nl = m2 * (m2 + 1) / 2, nw = m2 * (c + 1);
      // W entries: r0 = t m2 + (i - c - 2); (r0 + 1/2) / m2 is at least
      // 1/(2 m2) from an integer and the float product is within 2^-16 of
      // it, so the truncation gives t exactly (no integer division)
      const float inv_m2 = 1.0f / (float)m2;
      for (int q = tid - 64; q < nl + nw; q += POTF2_THREADS - 64) {
        if (q < nl) {
          const int r = tri_row[q];
          const int i = c + 2 + r, l = c + 2 + (q - r * (r + 1) / 2);
          const ddv p = dd_mul(ddv{lh[pk(i, c)], ll[pk(i, c)]}, ddv{lh[pk(l, c)], ll[pk(l, c)]});
          const ddv v = dd_add(ddv{lh[pk(i, l)], ll[pk(i, l)]}, dd_neg(p));
          lh[pk(i, l)] = v.hi;
          ll[pk(i, l)] = v.lo;
        } else {
          const int r0 = q - nl;
          const int t = (int)(((float)r0 + 0.5f) * inv_m2);
          const int i = c + 2 + (r0 - t * m2);
          const ddv p = dd_mul(ddv{lh[pk(i, c)], ll[pk(i, c)]}, ddv{wh[pk(c, t)], wl[pk(c, t)]});
          const ddv v = dd_add(ddv{wh[pk(i, t)], wl[pk(i, t)]}, dd_neg(p));
          wh[pk(i, t)] = v.hi;
          wl[pk(i, t)] = v.lo;
        }
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

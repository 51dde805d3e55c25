// ozaki.hip -- split-form dd Rgemm on the matrix cores of gfx950.
//
// The manual contains no split method; this is the error-free splitting of a
// matrix product (Ozaki, Ogita, Oishi, Rump 2012) in the integer-unit form of
// Ootomo, Ozaki and Yokota (2024), applied to dd operands:
//
//  scale    sigma_r = frexp exponent of max_l |x_rl.hi| for every row of op(A)
//           and every column of op(B) ("row operand"), so |x| < 2^sigma.
//  slice    y = x * 2^-sigma (exact); digit t: z = y * 2^w_t, q_t = rint(z.hi),
//           y = TwoSum(z.hi - q_t, z.lo).  INT8 form: w_1 = 6 and w_t = 8 while
//           nslices*k < 2^17 (a later digit that rounds to 128, or reaches it
//           by a carry, loses 256 and the digit before it gains one, so every
//           later digit is in [-128, 127]), else w_t = 7 (|q| <= 64); FP64
//           form: w_1 = w - 1, w_t = w with w chosen so that every sum of
//           nslices*k digit products stays an integer < 2^53.  Digits are
//           stored k-contiguous per row, in tiles padded with zeros.
//  products for every anti-diagonal d = t + u (2 <= d <= s + 1):
//           X_d = sum_t Q_t Q'_{d-t}^T, exact: int8 x int8 -> int32 on the
//           INT8 MFMA (|X_d| <= s*k*2^(2w-2) < 2^31), or FP64 MFMA on integers.
//  combine  P = sum_d X_d 2^-(2 w_1 + w (d-2)), added in dd (DWPlusFP) from the
//           smallest weight up; P * 2^(sigma_i + tau_j); C = alpha*P + beta*C.
// Binary64 arithmetic appears only in scaling, slicing and combining.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "../../include/mpdd.h"
#include "dd.hpp"
#include "crt.hpp"
#include "kernels.hpp"
#include "qd.hpp"

#pragma clang fp contract(off)

namespace mpdd {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// Tile geometry of the FP64 product kernel; slice buffers are padded to the
// product kernel's tile.
constexpr int OZ_BM = 128;      // rows of op(A) per workgroup tile (FP64 form)
constexpr int OZ_BN = 128;      // columns of op(B) per workgroup tile (FP64 form)
constexpr int OZ_KPAD = 64;     // k padding of the slice rows

// ---- scale -------------------------------------------------------------------------

// Row operand element (r, l) lives at x[r*sr + l*sl].  Rows contiguous across
// lanes (sr == 1): a workgroup takes 64 rows x one chunk of OZ_SCALE_CHUNK
// columns; lane r%64 of wave w reads columns w, w+4, ... of the chunk (each
// wave load is 64 consecutive doubles), the 4 waves' maxima meet in LDS, and
// the chunk maximum goes to part[chunk][row].  oz_scale_finish reduces the
// chunks and takes the frexp exponent.
constexpr int OZ_SCALE_CHUNK = 512;

__global__ void __launch_bounds__(256)
oz_scale_part_cols(const double* __restrict__ x, const double* __restrict__ x2, int64_t sr,
                   int64_t sl, int64_t rows, int64_t k, double* __restrict__ part) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  const int64_t l0 = (int64_t)blockIdx.y * OZ_SCALE_CHUNK;
  const int64_t l1 = (l0 + OZ_SCALE_CHUNK < k) ? l0 + OZ_SCALE_CHUNK : k;
  double mx = 0.0;
  if (r < rows) {
    for (int64_t l = l0 + wave; l < l1; l += 4) mx = fmax(mx, fabs(x[r * sr + l * sl]));
    if (x2)
      for (int64_t l = l0 + wave; l < l1; l += 4) mx = fmax(mx, fabs(x2[r * sr + l * sl]));
  }
  red[wave][lane] = mx;
  __syncthreads();
  if (wave == 0 && r < rows) {
    mx = fmax(fmax(red[0][lane], red[1][lane]), fmax(red[2][lane], red[3][lane]));
    part[(int64_t)blockIdx.y * rows + r] = mx;
  }
}

__global__ void __launch_bounds__(256)
oz_scale_finish(const double* __restrict__ part, int64_t rows, int nchunks,
                int* __restrict__ exps) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double mx = 0.0;
  for (int c = 0; c < nchunks; ++c) mx = fmax(mx, part[(int64_t)c * rows + r]);
  int e = 0;
  if (mx != 0.0) frexp(mx, &e);
  exps[r] = e;
}

// Rows contiguous along l (sl == 1): one wave per row, lanes walk l.
// x2 (may be null): a second plane whose entries count as well (the
// imaginary parts of a complex row operand).
__global__ void __launch_bounds__(256)
oz_scale_rows_wave(const double* __restrict__ x, const double* __restrict__ x2, int64_t sr,
                   int64_t sl, int64_t rows, int64_t k, int* __restrict__ exps) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (r >= rows) return;
  double mx = 0.0;
  for (int64_t l = lane; l < k; l += 64) mx = fmax(mx, fabs(x[r * sr + l * sl]));
  if (x2)
    for (int64_t l = lane; l < k; l += 64) mx = fmax(mx, fabs(x2[r * sr + l * sl]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if (lane == 0) {
    int e = 0;
    if (mx != 0.0) frexp(mx, &e);
    exps[r] = e;
  }
}

// ---- slice -------------------------------------------------------------------------

// One 64 x 64 block of the row operand per workgroup of 512 threads.
// Elements of both planes are read with lanes along whichever index is
// contiguous in memory and staged in LDS; then each thread turns 4
// consecutive l of two rows (8-bit digits kept in registers: one 4-byte
// store per digit, 16 threads store a row's 64 digits of a slice together)
// or 8 consecutive l of one row (the other forms: 8 int8 or 8 doubles per
// digit) into digits and writes them k-contiguously.  Rows >= rows and
// l >= k (padding) get zero digits.
//
// 8-bit int8 digits: a later digit of 128 does not fit, so it is carried into
// the digit before it (it loses 2^w = 256, that digit gains one; the value
// does not change).  A carry can turn a 127 into 128, so it runs on through
// digits of 127: a digit of 128 carries out, and so does each 127 directly
// before it in a run that ends in 128; any other digit ends the run.  With at
// most 16 digits the raw digits of an element stay in registers and every
// carry is known once its last digit is: digit t is then stored as
// raw_t + carry_in_t wrapped to 8 bits (a carried 128 + c becomes c - 128, a
// carried 127 + 1 becomes -128, the others do not wrap).  Longer digit
// strings take two passes: the first finds the carries, the second recomputes
// the digits and stores them carried.
//
// The remainder after a digit, (z.hi - q) + z.lo, is formed with FastTwoSum:
// z.hi - q is exact and a whole multiple of ulp(z.hi) (q is an integer, and
// |z.hi - q| <= 1/2 keeps it within z.hi's binade or below), so it is zero or
// at least ulp(z.hi) in magnitude, while |z.lo| <= ulp(z.hi)/2 for a
// normalised pair -- FastTwoSum's condition holds and it returns the same
// pair as TwoSum in half the operations.
constexpr int OZ_SLICE_REG_DIGITS = 16;

template <typename T>
__global__ void __launch_bounds__(512, 2)
oz_slice(const double* __restrict__ xh, const double* __restrict__ xl, int64_t sr, int64_t sl,
         int64_t rows, int64_t k, const int* __restrict__ exps, int nslices, int wfirst, int w,
         T* __restrict__ q, int64_t ldq, int64_t plane) {
  // staging for the hi and the lo plane (66.5 KB: two workgroups fit a CU),
  // so that both planes' loads are in flight together
  __shared__ double t[2][64][65];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * 64;
  const int64_t l0 = (int64_t)blockIdx.x * 64;
  const bool lanes_on_r = (sr == 1);
  const int rr = tid >> 3;
  const int lb = (tid & 7) * 8;
  const int64_t r = r0 + rr;
  const int e = (r < rows) ? exps[r] : 0;
  {
    double v[2][8];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const double* __restrict__ src = half ? xl : xh;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int a = tid & 63, b = (tid >> 6) + 8 * c;
        const int ri = lanes_on_r ? a : b;
        const int li = lanes_on_r ? b : a;
        const int64_t rg = r0 + ri, lg = l0 + li;
        v[half][c] = (rg < rows && lg < k) ? src[rg * sr + lg * sl] : 0.0;
      }
    }
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int a = tid & 63, b = (tid >> 6) + 8 * c;
        t[half][lanes_on_r ? a : b][lanes_on_r ? b : a] = v[half][c];
      }
  }
  __syncthreads();
  // scaled element i of this thread's 8 (the staging is not written again)
  auto scaled = [&](int i) {
    return ddv{ldexp(t[0][rr][lb + i], -e), ldexp(t[1][rr][lb + i], -e)};
  };
  T* out = q + r * ldq + l0 + lb;
  const bool carry = sizeof(T) == 1 && w > 7;

  if constexpr (sizeof(T) == 1) {
    if (carry && nslices <= OZ_SLICE_REG_DIGITS) {
      // here a thread takes 4 consecutive l of two rows, rq and rq + 32, so
      // that the 16 threads of a row store its 64 digits of a slice in one
      // contiguous piece; fw[t]: carried digit t of the 4 elements, one byte
      // each (one 4-byte store per digit)
      const int rq = tid >> 4, lq = (tid & 15) * 4;
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int row = rq + 32 * g;
        const int eg = (r0 + row < rows) ? exps[r0 + row] : 0;
        uint32_t fw[OZ_SLICE_REG_DIGITS];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ddv z{ldexp(t[0][row][lq + i], -eg), ldexp(t[1][row][lq + i], -eg)};
          int raw[OZ_SLICE_REG_DIGITS];
          uint32_t run = 0, cm = 0;              // bit t of cm: carry out of digit t
#pragma unroll
          for (int d = 0; d < OZ_SLICE_REG_DIGITS; ++d) {
            raw[d] = 0;
            if (d < nslices) {
              const int shift = (d == 0) ? wfirst : w;
              const double zh = ldexp(z.hi, shift), zl = ldexp(z.lo, shift);
              const double qd = rint(zh);
              z = fast_two_sum(zh - qd, zl);
              raw[d] = (int)qd;
              if (d > 0) {
                const uint32_t bit = 1u << d;
                if (raw[d] >= 128) {
                  cm |= run | bit;
                  run = 0;
                } else if (raw[d] == 127) {
                  run |= bit;
                } else {
                  run = 0;
                }
              }
            }
          }
#pragma unroll
          for (int d = 0; d < OZ_SLICE_REG_DIGITS; ++d) {
            const uint32_t byte = (uint32_t)(raw[d] + (int)((cm >> (d + 1)) & 1u)) & 0xFFu;
            if (i == 0)
              fw[d] = byte;
            else
              fw[d] |= byte << (8 * i);
          }
        }
        T* o = q + (r0 + row) * ldq + l0 + lq;
#pragma unroll
        for (int d = 0; d < OZ_SLICE_REG_DIGITS; ++d)
          if (d < nslices) *(uint32_t*)(o + (int64_t)d * plane) = fw[d];
      }
      return;
    }
  }

  ddv y[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) y[i] = scaled(i);
  // (longer 8-bit digit strings) first pass: the carries; bit d of cm[i] is
  // the carry out of digit d of element i
  uint64_t cm[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) cm[i] = 0;
  if (carry) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      ddv z = y[i];
      uint64_t run = 0, c = 0;
      for (int d = 0; d < nslices; ++d) {
        const int shift = (d == 0) ? wfirst : w;
        const double zh = ldexp(z.hi, shift), zl = ldexp(z.lo, shift);
        const double qd = rint(zh);
        z = fast_two_sum(zh - qd, zl);
        if (d == 0) continue;
        const uint64_t bit = (uint64_t)1 << d;
        if (qd >= 128.0) {
          c |= run | bit;
          run = 0;
        } else if (qd == 127.0) {
          run |= bit;
        } else {
          run = 0;
        }
      }
      cm[i] = c;
    }
  }
  for (int d = 0; d < nslices; ++d) {
    const int shift = (d == 0) ? wfirst : w;
    T dig[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double zh = ldexp(y[i].hi, shift), zl = ldexp(y[i].lo, shift);
      const double qd = rint(zh);
      // carry in from digit d + 1, carry out of digit d
      const int cin = (int)((cm[i] >> (d + 1)) & 1), cout = (int)((cm[i] >> d) & 1);
      dig[i] = (sizeof(T) == 1) ? (T)((int)qd + cin - (cout << w)) : (T)qd;
      y[i] = fast_two_sum(zh - qd, zl);
    }
    T* o = out + (int64_t)d * plane;
    if constexpr (sizeof(T) == 1) {
      uint2 pack;
      pack.x = (uint32_t)(uint8_t)dig[0] | ((uint32_t)(uint8_t)dig[1] << 8) |
               ((uint32_t)(uint8_t)dig[2] << 16) | ((uint32_t)(uint8_t)dig[3] << 24);
      pack.y = (uint32_t)(uint8_t)dig[4] | ((uint32_t)(uint8_t)dig[5] << 8) |
               ((uint32_t)(uint8_t)dig[6] << 16) | ((uint32_t)(uint8_t)dig[7] << 24);
      *(uint2*)o = pack;
    } else {
#pragma unroll
      for (int i = 0; i < 8; i += 2) *(double2*)(o + i) = double2{dig[i], dig[i + 1]};
    }
  }
}

// Largest y with y (y + 1) / 2 <= t.
__device__ __forceinline__ int oz_tri_root(int t) {
  int y = (int)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((y + 1) * (y + 2) / 2 <= t) ++y;
  while (y * (y + 1) / 2 > t) --y;
  return y;
}

// Tiles of one anti-diagonal group: the whole tiles_m x tiles_n grid, or for
// a triangle (tri 1: upper, tile row <= tile column; 2: lower; square
// tiles, tiles_m == tiles_n) only the tiles_m (tiles_m + 1) / 2 tiles that
// meet it.
__host__ __device__ __forceinline__ int oz_group_tiles(int tri, int tiles_m, int tiles_n) {
  return tri ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
}

// Workgroup b -> (anti-diagonal d, C tile (bi, bj)).  Groups of
// oz_group_tiles workgroups share one d, largest d (longest sum) first.
// Inside a group, each of the 8 XCDs (workgroups are dealt to them
// round-robin) receives a contiguous run of the tile sequence, and that
// sequence walks the C grid in 8 x 8 super-tiles (bi fastest inside one):
// the workgroups an XCD runs at the same time then cover a compact block of
// C and read a few row panels of op(A) and column panels of op(B), which its
// L2 holds, instead of every row panel of op(A) against one column panel.
// A triangle with tiles_m a multiple of 8 is walked in the same 8 x 8
// blocks: first the blocks off the diagonal (64 tiles each, blocks column by
// column), then the diagonal blocks (their 36 tiles each), so that every
// XCD's run holds an equal number of tiles; other triangles column by column.
__device__ __forceinline__ void oz_tile_of(int b, int tri, int tiles_m, int tiles_n, int nslices,
                                           int& d, int& bi, int& bj) {
  const int tiles = oz_group_tiles(tri, tiles_m, tiles_n);
  d = nslices + 1 - b / tiles;
  int r = b % tiles;
  if ((tiles & 7) == 0) r = (r & 7) * (tiles >> 3) + (r >> 3);
  if (tri) {
    int x, y;                                  // tile (x, y) with x <= y
    if ((tiles_m & 7) == 0) {
      const int s8 = tiles_m >> 3, off = 64 * (s8 * (s8 - 1) / 2);
      if (r < off) {
        const int by = oz_tri_root(r >> 6) + 1, bx = (r >> 6) - by * (by - 1) / 2;
        x = bx * 8 + (r & 7);
        y = by * 8 + ((r >> 3) & 7);
      } else {
        const int db = (r - off) / 36, w = (r - off) % 36;
        const int yy = oz_tri_root(w);
        x = db * 8 + (w - yy * (yy + 1) / 2);
        y = db * 8 + yy;
      }
    } else {
      y = oz_tri_root(r);
      x = r - y * (y + 1) / 2;
    }
    bi = (tri == 1) ? x : y;
    bj = (tri == 1) ? y : x;
    return;
  }
  if ((tiles_m & 7) == 0 && (tiles_n & 7) == 0) {
    const int st = r >> 6, w = r & 63, stm = tiles_m >> 3;
    bi = (st % stm) * 8 + (w & 7);
    bj = (st / stm) * 8 + (w >> 3);
  } else {
    bi = r % tiles_m;
    bj = r / tiles_m;
  }
}

// ---- products: INT8 ---------------------------------------------------------------------

// Four consecutive entries (rows i..i+3 of one column) of a residue product,
// |X| < 2^31, reduced modulo m: X (1/m) is within 2^-29 of X/m, so rint gives
// the nearest integer and X - q m (one exact fma) is the balanced residue (for
// m = 256 possibly +128, whose byte is that of -128: the same class).  One
// 4-byte store of the four int8 residues.
__device__ __forceinline__ void crt_store4(int8_t* p, int v0, int v1, int v2, int v3, double m,
                                           double minv) {
  auto red = [&](int v) {
    const double xv = (double)v;
    return (uint32_t)(int)fma(-rint(xv * minv), m, xv) & 0xFFu;
  };
  *(uint32_t*)p = red(v0) | (red(v1) << 8) | (red(v2) << 16) | (red(v3) << 24);
}

// X_d tile (WM x WN) for anti-diagonal d: sum over t of Q_t(rows) Q'_{d-t}(cols)^T
// with k-contiguous int8 rows.  GM x GN waves; each wave owns (WM/GM) x (WN/GN)
// outputs = (WM/GM/16) x (WN/GN/16) v_mfma_i32_16x16x64_i8
// tiles (int32 accumulators, held in AGPRs when they do not fit beside the
// fragments), so each 16-byte LDS fragment feeds several MFMAs.  A stage holds
// a W x 64-byte block of each operand in LDS (double buffered; 16-byte chunks
// XOR-permuted per row, i8_lds, so stores and fragment reads avoid bank
// conflicts).
// For an MFMA, lane l supplies row l % 16, bytes 16*(l/16) .. +15 of the
// k-step, for both operands, so every k pairs up.  Accumulation is exact in
// int32.  Variants (selected by mpdd_opts.tile_id for the INT8 form):
//   0: 256 x 256, 2 x 2 waves (128 x 128 each, 1 workgroup per CU)
//   1: 256 x 128, 2 x 2 waves (128 x 64 each, 2 workgroups per CU)
//   2: 128 x 128, 2 x 2 waves (64 x 64 each, 3 workgroups per CU)
//   3: 256 x 256, 2 x 4 waves (128 x 64 each, 512 threads: 2 waves per SIMD)
//   4: 256 x 256, 4 x 4 waves (64 x 64 each, 1024 threads: 4 waves per SIMD)
//   5, 6: the tiling of 3 in oz_gemm_i8_dma below (6 is the default)
//   7: 256 x 256, 2 x 2 waves in oz_gemm_i8_dma (1 wave per SIMD)
//   8: as 6 with v_mfma_i32_32x32x32_i8 (4 x 2 tiles of 32 x 32 per wave)
constexpr int I8_BK = 64;
constexpr int I8_PITCH = 64;   // bytes per staged row (one k-step), no padding

// LDS position of 16-byte chunk c of staged row r: chunks are permuted by an
// XOR with ((r >> 1) ^ (r >> 2)) & 3, so that both the staging stores (each 8
// or 16 lanes write 2 or 4 whole rows) and the fragment reads (lanes l read
// chunk l / 16 of rows r0 + l % 16, r0 a multiple of 16) touch distinct banks
// whether the LDS serves 8 lanes per 128 bytes or 16 lanes per 256 bytes.
__device__ __forceinline__ int i8_lds(int r, int c) {
  return r * I8_PITCH + ((c ^ ((r >> 1) ^ (r >> 2))) & 3) * 16;
}
constexpr int I8_PAD = 256;     // slice rows are padded to this for every variant

template <int WM, int WN, int GM, int GN>
__global__ void __launch_bounds__(64 * GM * GN, (WM * WN / (GM * GN) > 128 * 64) ? 1 : (GM * GN > 8 ? 4 : 2))
oz_gemm_i8(const int8_t* __restrict__ qa, const int8_t* __restrict__ qb, int32_t* __restrict__ x,
           int64_t kp, int64_t plane_a, int64_t plane_b, int64_t mp, int64_t np, int nslices,
           int tiles_m, int tiles_n, int tri) {
  constexpr int NT = 64 * GM * GN;             // threads: a GM x GN grid of waves
  constexpr int WR = WM / GM, WC = WN / GN;    // outputs per wave
  constexpr int FA = WR / 16, FB = WC / 16;    // 16-row fragments per wave
  constexpr int SR = NT / 4;                   // rows staged per pass (4 threads per row)
  constexpr int EA = WM / SR, EB = WN / SR;    // 16-byte staging loads per thread
  static_assert(WM % SR == 0 && WN % SR == 0, "staging must cover the tile");
  __shared__ __attribute__((aligned(16))) int8_t As[2][WM * I8_PITCH];
  __shared__ __attribute__((aligned(16))) int8_t Bs[2][WN * I8_PITCH];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % GM, wn = wave / GM;

  int d, bi, bj;
  oz_tile_of(blockIdx.x, tri, tiles_m, tiles_n, nslices, d, bi, bj);
  const int64_t i0 = (int64_t)bi * WM, j0 = (int64_t)bj * WN;

  v4i acc[FA][FB];
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int c = 0; c < FB; ++c) acc[a][c] = v4i{0, 0, 0, 0};

  // staging: thread loads 16 bytes (chunk tid%4) of rows tid/4 + 64*e.  Global
  // loads run two k-steps ahead of the MFMAs (two register sets, used
  // alternately), so a load has two steps of matrix work to arrive before
  // its data is written to LDS.
  const int srow = tid >> 2, schunk = tid & 3, scol = schunk * 16;
  const int64_t ksteps = kp / I8_BK;
  const int64_t total = (int64_t)(d - 1) * ksteps;
  v4i ra0[EA], rb0[EB], ra1[EA], rb1[EB];

  auto gload = [&](int64_t s, v4i (&ra)[EA], v4i (&rb)[EB]) {
    const int t = 1 + (int)(s / ksteps);          // slice of op(A); op(B) slice d - t
    const int64_t l0 = (s % ksteps) * I8_BK;
    const int8_t* pa = qa + (int64_t)(t - 1) * plane_a + (i0 + srow) * kp + l0 + scol;
    const int8_t* pb = qb + (int64_t)(d - t - 1) * plane_b + (j0 + srow) * kp + l0 + scol;
#pragma unroll
    for (int e = 0; e < EA; ++e) ra[e] = *(const v4i*)(pa + SR * e * kp);
#pragma unroll
    for (int e = 0; e < EB; ++e) rb[e] = *(const v4i*)(pb + SR * e * kp);
  };
  auto sstore = [&](int buf, const v4i (&ra)[EA], const v4i (&rb)[EB]) {
#pragma unroll
    for (int e = 0; e < EA; ++e) *(v4i*)&As[buf][i8_lds(srow + SR * e, schunk)] = ra[e];
#pragma unroll
    for (int e = 0; e < EB; ++e) *(v4i*)&Bs[buf][i8_lds(srow + SR * e, schunk)] = rb[e];
  };
  const int fr = lane & 15, fc = lane >> 4;
  auto compute = [&](int cur) {
    v4i af[FA], bf[FB];
#pragma unroll
    for (int a = 0; a < FA; ++a)
      af[a] = *(const v4i*)&As[cur][i8_lds(wm * WR + a * 16 + fr, fc)];
#pragma unroll
    for (int c = 0; c < FB; ++c)
      bf[c] = *(const v4i*)&Bs[cur][i8_lds(wn * WC + c * 16 + fr, fc)];
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
      for (int c = 0; c < FB; ++c)
        acc[a][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[c], acc[a][c], 0, 0, 0);
  };

  // step s computes LDS buffer s & 1; even steps load into set 0 and store
  // set 1, odd steps the other way round.  kp is a multiple of 2 * I8_BK, so
  // the step count is even and both halves of every iteration run.
  gload(0, ra0, rb0);
  gload(1, ra1, rb1);
  sstore(0, ra0, rb0);
  __syncthreads();
  // (the loads and stores are unconditional, so that the wait counts are the
  // same on every iteration; past the end they re-read the last step, whose
  // data is stored but never used)
  for (int64_t s = 0; s < total; s += 2) {
    gload(s + 2 < total ? s + 2 : total - 1, ra0, rb0);
    // keep the loads ahead of the MFMAs (not for the 256 x 256 tile, whose
    // accumulators leave no room for the longer-lived staging registers)
    if constexpr (WR * WC <= 128 * 64) __builtin_amdgcn_sched_barrier(0);
    compute(0);
    sstore(1, ra1, rb1);
    __syncthreads();
    gload(s + 3 < total ? s + 3 : total - 1, ra1, rb1);
    if constexpr (WR * WC <= 128 * 64) __builtin_amdgcn_sched_barrier(0);
    compute(1);
    sstore(0, ra0, rb0);
    __syncthreads();
  }

  // C layout of a 16x16 INT8 MFMA tile: lane l holds rows 4*(l/16) + 0..3 of column l%16.
  int32_t* xd = x + (int64_t)(d - 2) * mp * np;
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int c = 0; c < FB; ++c) {
      const int64_t i = i0 + wm * WR + a * 16 + (lane >> 4) * 4;
      const int64_t j = j0 + wn * WC + c * 16 + (lane & 15);
      *(v4i*)&xd[j * mp + i] = acc[a][c];
    }
}

// Direct-to-LDS form of the same product (variant 5): the digits travel from
// global memory straight into LDS (global_load_lds_dwordx4: lane l of a wave
// writes 16 bytes at M0 + 16 l), so no registers stage them and no ds_write
// stores them.  NS stages form a ring; the loads of a stage are issued NS - 1
// steps before its matrix work, and one barrier per step both publishes the
// stage about to be used and frees the one about to be refilled.  A DMA
// instruction fills 16 staged rows (1 KB, the i8_lds layout); each lane picks
// the global chunk that the layout places at its slot, so the XOR permutation
// is applied on the global side.
// Wait until at most VM of this wave's global loads (here: LDS DMA) and LGKM
// of its LDS reads are outstanding, then meet the workgroup barrier.  One asm
// statement with a memory clobber, so that no LDS access moves across it.
template <int VM, int LGKM>
__device__ __forceinline__ void i8_sync() {
  static_assert(VM >= 0 && VM <= 63 && LGKM >= 0 && LGKM <= 15, "s_waitcnt fields");
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(%1)\n\ts_barrier" ::"n"(VM), "n"(LGKM) : "memory");
}

template <int WM, int WN, int GM, int GN, int NS, bool PF, bool M32, bool CRT = false>
__global__ void __launch_bounds__(64 * GM * GN, 1)
oz_gemm_i8_dma(const int8_t* __restrict__ qa, const int8_t* __restrict__ qb,
               int32_t* __restrict__ x, int64_t kp, int64_t plane_a, int64_t plane_b, int64_t mp,
               int64_t np, int nslices, int tiles_m, int tiles_n, int tri, CrtModuli cm,
               int crt_count, int crt_total, int crt_group) {
  constexpr int NW = GM * GN;                  // waves
  constexpr int WR = WM / GM, WC = WN / GN;    // outputs per wave
  constexpr int MT = M32 ? 32 : 16;            // MFMA tile edge
  constexpr int KS = M32 ? 2 : 1;              // MFMA k-slabs per 64-byte step
  constexpr int FA = WR / MT, FB = WC / MT;    // fragments per wave and slab
  constexpr int RA = WM / NW, RB = WN / NW;    // rows of each operand one wave stages
  constexpr int LA = RA / 16, LB = RB / 16;    // DMA instructions per operand and step
  constexpr int STAGE = (WM + WN) * I8_PITCH;  // bytes per stage
  static_assert(RA % 16 == 0 && RB % 16 == 0, "a DMA instruction stages 16 rows");
  __shared__ __attribute__((aligned(1024))) int8_t smem[NS * STAGE];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % GM, wn = wave / GM;

  int d, bi, bj;
  oz_tile_of(blockIdx.x, tri, tiles_m, tiles_n, nslices, d, bi, bj);
  // modular form: group d - 2 of crt_group consecutive residue planes; the
  // workgroup multiplies plane ct0 + g of both operands for each g in turn
  // (one k-sweep each, slice it - 1 of both operands below), storing each
  // product when its sweep ends
  int ct0 = 0;
  if constexpr (CRT) {
    ct0 = (d - 2) * crt_group;
    const int here = min(crt_group, crt_total - ct0);
    qa += (int64_t)ct0 * plane_a;
    qb += (int64_t)ct0 * plane_b;
    d = here + 1;
  }
  const int64_t i0 = (int64_t)bi * WM, j0 = (int64_t)bj * WN;

  typedef int v16i __attribute__((ext_vector_type(16)));
  typedef typename std::conditional<M32, v16i, v4i>::type accv;
  accv acc[FA][FB];
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int c = 0; c < FB; ++c) acc[a][c] = accv{};

  // lane l of a DMA instruction fills staged row r0 + l/4 (r0 a multiple of
  // 16), physical chunk l%4, which holds logical chunk (l%4) ^ g(row); g
  // depends only on the row's low four bits, i.e. on l/4
  const int lr = lane >> 2;
  const int lc = ((lane & 3) ^ (lr >> 1) ^ (lr >> 2)) & 3;
  const int64_t ksteps = kp / I8_BK;
  const int64_t total = (int64_t)(d - 1) * ksteps;
  const int8_t* ga = qa + (i0 + wave * RA + lr) * kp + lc * 16;
  const int8_t* gb = qb + (j0 + wave * RB + lr) * kp + lc * 16;

  // Steps are issued in order, step x into stage x % NS; (it, il0) is the
  // slice and k offset of the next one.  Steps past the end re-load the last
  // step (into a stage no later step reads), so that every step issues the
  // same loads and the wait counts are constants.
  int it = 1, ibuf = 0;
  int64_t il0 = 0, inext = 0;
  auto issue = [&]() {
    const int8_t* pa = ga + (int64_t)(it - 1) * plane_a + il0;
    // op(B) slice d - t (the modular form: the same plane as op(A))
    const int8_t* pb = gb + (int64_t)(CRT ? it - 1 : d - it - 1) * plane_b + il0;
    int8_t* st = smem + ibuf * STAGE;
#pragma unroll
    for (int e = 0; e < LA; ++e)
      __builtin_amdgcn_global_load_lds(
          (const void*)(pa + (int64_t)16 * e * kp),
          (__attribute__((address_space(3))) void*)(st + (wave * RA + 16 * e) * I8_PITCH), 16, 0,
          0);
#pragma unroll
    for (int e = 0; e < LB; ++e)
      __builtin_amdgcn_global_load_lds(
          (const void*)(pb + (int64_t)16 * e * kp),
          (__attribute__((address_space(3))) void*)(st + WM * I8_PITCH +
                                                    (wave * RB + 16 * e) * I8_PITCH),
          16, 0, 0);
    if (++inext < total) {
      il0 += I8_BK;
      if (il0 == kp) {
        il0 = 0;
        ++it;
      }
    }
    ibuf = (ibuf + 1 == NS) ? 0 : ibuf + 1;
  };
  // fragment row and 16-byte chunk of this lane: 16 x 16 x 64 MFMAs take
  // row l % 16, chunk l / 16; 32 x 32 x 32 ones take row l % 32, chunk
  // 2 h + l / 32 of k-slab h
  const int fr = lane & (MT - 1), fc = lane / MT;
  auto fetch = [&](int buf, v4i (&af)[KS * FA], v4i (&bf)[KS * FB]) {
    const int8_t* As = smem + buf * STAGE;
    const int8_t* Bs = As + WM * I8_PITCH;
#pragma unroll
    for (int h = 0; h < KS; ++h) {
#pragma unroll
      for (int a = 0; a < FA; ++a)
        af[h * FA + a] = *(const v4i*)&As[i8_lds(wm * WR + a * MT + fr, KS * h + fc)];
#pragma unroll
      for (int c = 0; c < FB; ++c)
        bf[h * FB + c] = *(const v4i*)&Bs[i8_lds(wn * WC + c * MT + fr, KS * h + fc)];
    }
  };
  auto mfma = [&](const v4i (&af)[KS * FA], const v4i (&bf)[KS * FB]) {
#pragma unroll
    for (int h = 0; h < KS; ++h)
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int c = 0; c < FB; ++c) {
          if constexpr (M32)
            acc[a][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[h * FA + a], bf[h * FB + c],
                                                              acc[a][c], 0, 0, 0);
          else
            acc[a][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[c], acc[a][c], 0, 0, 0);
        }
  };
  // The fragments read one step earlier have long arrived: waiting for them
  // (lgkmcnt(0), before the next prefetch is issued) costs nothing and tells
  // the compiler that the MFMAs need not wait for the prefetch.
  auto frags_landed = [&]() {
    __builtin_amdgcn_s_waitcnt(0xC07F);        // lgkmcnt(0); vmcnt, expcnt not waited on
    __builtin_amdgcn_sched_barrier(0);
  };
  // modular form: store the finished product of plane ct as int8 residues
  // modulo modulus ct % crt_count (a complex or qd product runs three products
  // per modulus, planes t, count + t, 2 count + t) and clear the accumulators
  // C layout: 16 x 16 tile, lane l holds rows 4 (l / 16) + 0..3 of column
  // l % 16; 32 x 32 tile, lane l holds rows 8 g + 4 (l / 32) + 0..3 of column
  // l % 32 in registers 4 g .. 4 g + 3
  auto crt_epilogue = [&](int ct) {
    int8_t* xq = (int8_t*)x + (int64_t)ct * mp * np;
    const int mt = ct % crt_count;
    const double mm = cm.m[mt], mi = cm.minv[mt];
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
      for (int c = 0; c < FB; ++c) {
        const int64_t j = j0 + wn * WC + c * MT + (lane & (MT - 1));
        if constexpr (M32) {
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int64_t i = i0 + wm * WR + a * MT + 8 * g + 4 * (lane >> 5);
            crt_store4(xq + j * mp + i, acc[a][c][4 * g], acc[a][c][4 * g + 1],
                       acc[a][c][4 * g + 2], acc[a][c][4 * g + 3], mm, mi);
          }
        } else {
          const int64_t i = i0 + wm * WR + a * MT + (lane >> 4) * 4;
          crt_store4(xq + j * mp + i, acc[a][c][0], acc[a][c][1], acc[a][c][2], acc[a][c][3],
                     mm, mi);
        }
        acc[a][c] = accv{};
      }
  };
  int64_t next_end = ksteps;                   // step count at which the current product ends
  int done = 0;                                // products of the group stored so far

  constexpr int PER = LA + LB;                 // DMA instructions per step and wave
  // LDS reads that may stay in flight at a barrier: the prefetch (FA + FB
  // reads), capped by the 4-bit counter (waiting for its oldest read as well
  // is harmless)
  constexpr int PFQ = (KS * (FA + FB) < 15) ? KS * (FA + FB) : 15;

#pragma unroll
  for (int q = 0; q < NS - 1; ++q) issue();
  if constexpr (!PF) {
    // step s: issued 0 .. s + NS - 2, so step s has landed once the loads of
    // NS - 2 later steps remain; no LDS read is in flight at the barrier (the
    // reads of step s - 1 fed its MFMAs), so stage (s - 1) % NS may be refilled
    for (int64_t s = 0; s < total; ++s) {
      i8_sync<(NS - 2) * PER, 0>();
      issue();                                 // step s + NS - 1
      v4i af[KS * FA], bf[KS * FB];
      fetch((int)(s % NS), af, bf);
      mfma(af, bf);
      if constexpr (CRT) {
        if (s + 1 == next_end && s + 1 < total) {
          crt_epilogue(ct0 + done++);
          next_end += ksteps;
        }
      }
    }
  } else {
    // fragments of step s + 1 are read from LDS while the MFMAs of step s run
    // (two register sets).  At step s, issued 0 .. s + NS - 2: step s + 1 has
    // landed once the loads of NS - 3 later steps remain; the LDS reads of the
    // prefetch of step s (FA + FB, the youngest) may still be in flight, those
    // of step s - 1 are done, so stage (s - 1) % NS may be refilled.
    static_assert(NS >= 4, "prefetch needs four stages");
    v4i af0[KS * FA], bf0[KS * FB], af1[KS * FA], bf1[KS * FB];
    i8_sync<(NS - 2) * PER, 0>();
    fetch(0, af0, bf0);
    // total is even (kp is a multiple of 2 * I8_BK)
    for (int64_t s = 0; s < total; s += 2) {
      i8_sync<(NS - 3) * PER, PFQ>();
      issue();                                 // step s + NS - 1
      frags_landed();
      fetch((int)((s + 1) % NS), af1, bf1);
      mfma(af0, bf0);
      // after the last pair this prefetches a stage no step uses: harmless
      i8_sync<(NS - 3) * PER, PFQ>();
      issue();                                 // step s + NS
      frags_landed();
      fetch((int)((s + 2) % NS), af0, bf0);
      mfma(af1, bf1);
      if constexpr (CRT) {
        // a sweep ends after an even step count (ksteps is even)
        if (s + 2 == next_end && s + 2 < total) {
          crt_epilogue(ct0 + done++);
          next_end += ksteps;
        }
      }
    }
  }
  // the loads past the end must land before the workgroup's LDS is released
  __builtin_amdgcn_s_waitcnt(0x0F70);          // vmcnt(0), lgkmcnt not waited on
  __builtin_amdgcn_sched_barrier(0);

  if constexpr (CRT) {
    crt_epilogue(ct0 + done);
    return;
  }
  int32_t* xd = x + (int64_t)(d - 2) * mp * np;
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int c = 0; c < FB; ++c) {
      const int64_t j = j0 + wn * WC + c * MT + (lane & (MT - 1));
      if constexpr (M32) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int64_t i = i0 + wm * WR + a * MT + 8 * g + 4 * (lane >> 5);
          *(v4i*)&xd[j * mp + i] = v4i{acc[a][c][4 * g], acc[a][c][4 * g + 1],
                                       acc[a][c][4 * g + 2], acc[a][c][4 * g + 3]};
        }
      } else {
        const int64_t i = i0 + wm * WR + a * MT + (lane >> 4) * 4;
        *(v4i*)&xd[j * mp + i] = acc[a][c];
      }
    }
}

// ---- products: FP64 ---------------------------------------------------------------------

// Same tiling with v_mfma_f64_16x16x4_f64: a k-step stages 16 doubles per row;
// lane l supplies row l % 16 at k-offset l / 16 of each 4-deep MFMA.  Digit
// products and all their partial sums are integers below 2^53, so the FP64
// accumulation is exact in any order.
constexpr int F64_BK = 16;
constexpr int F64_PITCH = 17;

__global__ void __launch_bounds__(256)
oz_gemm_f64(const double* __restrict__ qa, const double* __restrict__ qb, double* __restrict__ x,
            int64_t kp, int64_t plane_a, int64_t plane_b, int64_t mp, int64_t np, int nslices,
            int tiles_m, int tiles_n, int tri) {
  __shared__ double As[2][OZ_BM * F64_PITCH];
  __shared__ double Bs[2][OZ_BN * F64_PITCH];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  int d, bi, bj;
  oz_tile_of(blockIdx.x, tri, tiles_m, tiles_n, nslices, d, bi, bj);
  const int64_t i0 = (int64_t)bi * OZ_BM, j0 = (int64_t)bj * OZ_BN;

  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = v4d{0.0, 0.0, 0.0, 0.0};

  // staging: 128 rows x 16 doubles per operand = 2048 doubles; 8 per thread:
  // thread handles row (tid / 2) and 8 consecutive k at (tid % 2) * 8.
  const int srow = tid >> 1, scol = (tid & 1) * 8;
  const int64_t ksteps = kp / F64_BK;
  const int64_t total = (int64_t)(d - 1) * ksteps;
  double ra[8], rb[8];

  auto gload = [&](int64_t s) {
    const int t = 1 + (int)(s / ksteps);
    const int64_t l0 = (s % ksteps) * F64_BK;
    const double* pa = qa + (int64_t)(t - 1) * plane_a + (i0 + srow) * kp + l0 + scol;
    const double* pb = qb + (int64_t)(d - t - 1) * plane_b + (j0 + srow) * kp + l0 + scol;
#pragma unroll
    for (int e = 0; e < 8; ++e) { ra[e] = pa[e]; rb[e] = pb[e]; }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[buf][srow * F64_PITCH + scol + e] = ra[e];
      Bs[buf][srow * F64_PITCH + scol + e] = rb[e];
    }
  };

  gload(0);
  sstore(0);
  __syncthreads();
  const int fr = lane & 15, fk = lane >> 4;
  for (int64_t s = 0; s < total; ++s) {
    const int cur = (int)(s & 1);
    if (s + 1 < total) gload(s + 1);
#pragma unroll
    for (int kk = 0; kk < F64_BK; kk += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) af[a] = As[cur][(wm * 64 + a * 16 + fr) * F64_PITCH + kk + fk];
#pragma unroll
      for (int c = 0; c < 4; ++c) bf[c] = Bs[cur][(wn * 64 + c * 16 + fr) * F64_PITCH + kk + fk];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[c], acc[a][c], 0, 0, 0);
    }
    if (s + 1 < total) sstore(cur ^ 1);
    __syncthreads();
  }

  // C layout of the FP64 16x16 MFMA tile: lane l, register e holds row
  // 4*e + l/16 of column l%16 (unlike the INT8 form's 4*(l/16) + e).
  double* xd = x + (int64_t)(d - 2) * mp * np;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t i = i0 + wm * 64 + a * 16 + (lane >> 4);
      const int64_t j = j0 + wn * 64 + c * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) xd[j * mp + i + 4 * e] = acc[a][c][e];
    }
}

// ---- combine -------------------------------------------------------------------------

// Four consecutive rows i0 .. i0+3 of one column j per thread (for a
// triangle, only its entries are read and written): each
// anti-diagonal sum is one 16-byte (int32) or 32-byte (fp64) load per thread
// (plane rows are padded to a multiple of 256, so the four are in range and
// aligned); the C entries (when read) are loaded first and a batch of NB
// anti-diagonals (8 int32, 4 fp64) is loaded before any is added, so that
// many loads are in flight at once.  Per entry the steps are the same as one
// entry at a time: smallest weight first (d = nslices+1 down to 2),
// DWPlusFP, then the scale and alpha / beta.
template <typename XT>
__global__ void __launch_bounds__(256)
oz_combine(const XT* __restrict__ x, int64_t mp, int64_t np, int nslices, int wfirst, int w,
           const int* __restrict__ ea, const int* __restrict__ eb, int64_t m, int64_t n,
           double alpha_hi, double alpha_lo, double beta_hi, double beta_lo, int beta_zero,
           double* __restrict__ c_hi, double* __restrict__ c_lo, int64_t ldc, int tri) {
  typedef XT xv4 __attribute__((ext_vector_type(4)));
  constexpr int NB = sizeof(XT) == 4 ? 8 : 4;
  const int64_t mq = (m + 3) / 4;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= mq * n) return;
  const int64_t i0 = (gid % mq) * 4, j = gid / mq;
  // rows of column j that are updated: all, or the triangle's (tri 1:
  // upper, i <= j; 2: lower, i >= j); a thread with none of them returns
  // before reading anything (its tile may not have been computed)
  const int64_t ilo = (tri == 2) ? j : 0, ihi = (tri == 1) ? j : m - 1;
  if (i0 > ihi || i0 + 3 < ilo) return;
  auto updated = [&](int64_t i) { return i < m && i >= ilo && i <= ihi; };
  const XT* xp = x + j * mp + i0;
  const int64_t plane = mp * np;
  double ch[4] = {0.0, 0.0, 0.0, 0.0}, cl[4] = {0.0, 0.0, 0.0, 0.0};
  if (!beta_zero) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (updated(i0 + r)) {
        ch[r] = c_hi[i0 + r + j * ldc];
        cl[r] = c_lo[i0 + r + j * ldc];
      }
  }
  ddv p[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) p[r] = ddv{0.0, 0.0};
  for (int d0 = nslices + 1; d0 >= 2; d0 -= NB) {
    xv4 v[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u)
      v[u] = d0 - u >= 2 ? *(const xv4*)(xp + (int64_t)(d0 - u - 2) * plane) : xv4{0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (d0 - u < 2) continue;
      const int sh = -(2 * wfirst + w * (d0 - u - 2));
#pragma unroll
      for (int r = 0; r < 4; ++r) p[r] = dd_add_d(p[r], ldexp((double)v[u][r], sh));
    }
  }
  const ddv alpha{alpha_hi, alpha_lo}, beta{beta_hi, beta_lo};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t i = i0 + r;
    if (!updated(i)) continue;
    const int e = ea[i] + eb[j];
    ddv pr{ldexp(p[r].hi, e), ldexp(p[r].lo, e)};
    ddv res = dd_mul(alpha, pr);
    const int64_t ci = i + j * ldc;
    if (!beta_zero) res = dd_add(res, dd_mul(beta, ddv{ch[r], cl[r]}));
    c_hi[ci] = res.hi;
    c_lo[ci] = res.lo;
  }
}

// ---- split form for quad-double operands -------------------------------------------

// Slices of a row operand of quad-doubles (x0 + x1 + x2 + x3, four planes),
// INT8 digits only.  Staging as in oz_slice (one 33 KB buffer, each part in
// turn); each thread then turns 8 consecutive l of one row into digits.
// Digit t: z = y 2^w_t (exact), q_t = rint(z0), z0 - q_t (exact), then two
// TwoSum sweeps renormalise the four parts: every TwoSum is error-free, so
// the remainder stays exact, and after the bottom-up sweep z0 is the
// rounded value of the remainder with the rest below about ulp(z0), which
// keeps the next digit within the balanced range of oz_slice.  8-bit digits
// are carried as there, in two passes (the carries first; digit strings up
// to 64 long); 7-bit digits need no carries.
constexpr int OZ_QD_MAX_SLICES = 48;

__global__ void __launch_bounds__(512)
oz_slice_qd(const double* __restrict__ x0, const double* __restrict__ x1,
            const double* __restrict__ x2, const double* __restrict__ x3, int64_t sr, int64_t sl,
            int64_t rows, int64_t k, const int* __restrict__ exps, int nslices, int wfirst, int w,
            int8_t* __restrict__ q, int64_t ldq, int64_t plane) {
  __shared__ double t[64][65];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * 64;
  const int64_t l0 = (int64_t)blockIdx.x * 64;
  const bool lanes_on_r = (sr == 1);
  const int rr = tid >> 3;
  const int lb = (tid & 7) * 8;
  const int64_t r = r0 + rr;
  const int e = (r < rows) ? exps[r] : 0;
  qacc y[8];
#pragma unroll
  for (int part = 0; part < 4; ++part) {
    const double* __restrict__ src = part == 0 ? x0 : part == 1 ? x1 : part == 2 ? x2 : x3;
    double v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int a = tid & 63, b = (tid >> 6) + 8 * c;
      const int ri = lanes_on_r ? a : b;
      const int li = lanes_on_r ? b : a;
      const int64_t rg = r0 + ri, lg = l0 + li;
      v[c] = (rg < rows && lg < k) ? src[rg * sr + lg * sl] : 0.0;
    }
    if (part) __syncthreads();                 // the previous part has been read
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int a = tid & 63, b = (tid >> 6) + 8 * c;
      t[lanes_on_r ? a : b][lanes_on_r ? b : a] = v[c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double xv = ldexp(t[rr][lb + i], -e);
      if (part == 0) y[i].s0 = xv;
      else if (part == 1) y[i].s1 = xv;
      else if (part == 2) y[i].s2 = xv;
      else y[i].s3 = xv;
    }
  }
  // one digit of z (in place: z becomes the remainder)
  auto digit = [](qacc& z, int shift) -> int {
    z.s0 = ldexp(z.s0, shift);
    z.s1 = ldexp(z.s1, shift);
    z.s2 = ldexp(z.s2, shift);
    z.s3 = ldexp(z.s3, shift);
    const double qd = rint(z.s0);
    z.s0 = z.s0 - qd;
    qd_renorm(z);
    return (int)qd;
  };
  // bit d of cm[i]: the carry out of digit d of element i (8-bit digits)
  uint64_t cm[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) cm[i] = 0;
  if (w > 7) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      qacc z = y[i];
      uint64_t run = 0, c = 0;
      for (int d = 0; d < nslices; ++d) {
        const int qv = digit(z, d == 0 ? wfirst : w);
        if (d == 0) continue;
        const uint64_t bit = (uint64_t)1 << d;
        if (qv >= 128) {
          c |= run | bit;
          run = 0;
        } else if (qv == 127) {
          run |= bit;
        } else {
          run = 0;
        }
      }
      cm[i] = c;
    }
  }
  int8_t* out = q + r * ldq + l0 + lb;
  for (int d = 0; d < nslices; ++d) {
    const int shift = (d == 0) ? wfirst : w;
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int qv = digit(y[i], shift);
      const int cin = (int)((cm[i] >> (d + 1)) & 1), cout = (int)((cm[i] >> d) & 1);
      const uint32_t byte = (uint32_t)(qv + cin - (cout << w)) & 0xFFu;
      if (i < 4)
        lo |= byte << (8 * i);
      else
        hi |= byte << (8 * (i - 4));
    }
    *(uint2*)(out + (int64_t)d * plane) = uint2{lo, hi};
  }
}

// qd combine: one output (i, j) per thread.  The anti-diagonal sums are
// added in qd from the smallest weight up (each X_d 2^-e_d is an exact
// binary64: TwoSum into the leading part, the errors passed down the
// levels, renormalised), then the exact power-of-two scale, then
// C = alpha P + beta C as qd products by levels (beta = 0: C not read).
__global__ void __launch_bounds__(256)
oz_combine_qd(const int32_t* __restrict__ x, int64_t mp, int64_t np, int nslices, int wfirst,
              int w, const int* __restrict__ ea, const int* __restrict__ eb, int64_t m, int64_t n,
              double4 alpha, double4 beta, int beta_zero, double* __restrict__ c0,
              double* __restrict__ c1, double* __restrict__ c2, double* __restrict__ c3,
              int64_t ldc) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= m * n) return;
  const int64_t i = gid % m, j = gid / m;
  const int64_t plane = mp * np;
  const int32_t* xp = x + j * mp + i;
  qacc p{0.0, 0.0, 0.0, 0.0};
  for (int d = nslices + 1; d >= 2; --d) {
    const double v = ldexp((double)xp[(int64_t)(d - 2) * plane], -(2 * wfirst + w * (d - 2)));
    double e;
    ts(p.s0, v, p.s0, e);
    ts(p.s1, e, p.s1, e);
    ts(p.s2, e, p.s2, e);
    p.s3 = p.s3 + e;
    qd_renorm(p);
  }
  const double4 pf = qd_final(p);
  const int sc = ea[i] + eb[j];
  const double4 ps{ldexp(pf.x, sc), ldexp(pf.y, sc), ldexp(pf.z, sc), ldexp(pf.w, sc)};
  const int64_t ci = i + j * ldc;
  qacc r{0.0, 0.0, 0.0, 0.0};
  qd_madd(r, alpha, ps);
  if (!beta_zero) {
    qd_renorm(r);
    qd_madd(r, beta, double4{c0[ci], c1[ci], c2[ci], c3[ci]});
  }
  const double4 o = qd_final(r);
  c0[ci] = o.x;
  c1[ci] = o.y;
  c2[ci] = o.z;
  c3[ci] = o.w;
}

// ---- modular split form ------------------------------------------------------------

// Residues of a row operand.  Element x of row r becomes the integer
// x' = t1 + t2 on the grid of P bits below 2^sigma_r: z = x 2^(P - sigma_r)
// (exact, zh + zl), t1 = rint(zh), t2 = rint((zh - t1) + zl), |x'| <= 2^P.
// Plane t (0-based) receives x' modulo modulus t, balanced (odd m: in
// [-(m-1)/2, (m-1)/2]; m = 256: the low byte), as int8 at
// q + t*plane + r*ldq + l; padding rows and columns get 0.
//
// x' is handled in 26-bit chunks: t1 = u 2^52 + v (u = rint(t1 2^-52); v is
// an integer with |v| <= 2^51, so the fma that forms it is exact),
// w = v + t2 (exact: |w| < 2^53 while P <= 104), u = u1 2^26 + u0 and
// w = w1 2^26 + w0 (|u0|, |w0| <= 2^25).  Then x' = u1 2^78 + u0 2^52 +
// w1 2^26 + w0, and y = u1 c78 + u0 c52 + w1 c26 + w0 (c_j = 2^j mod m) is
// congruent to x' and below 2^37 in magnitude, exact in binary64.  For odd m,
// y/m lies at least 1/(2m) from a half-integer while y * (1/m) is within
// 2^-23 of it, so q = rint(y * (1/m)) is the nearest integer and y - q m
// (one exact fma) the balanced residue.  m = 256 is plane 0: the low byte of
// w0 (w0 = x' modulo 2^26).
//
// A workgroup takes a block of 32 rows x 128 l: both planes are loaded with
// lanes along the contiguous index and staged in LDS (74 KB: two workgroups
// per CU); each thread then converts 8 consecutive l of one row and stores
// one 8-byte word per modulus, so the 16 threads of a row write its 128
// residues of a plane as one 128-byte line.  Columns l >= ldq (ldq is a
// multiple of 64) are neither stored nor, beyond k, read.
//
// Complex operands: sign = -1 negates every entry (a conjugated imaginary
// part; the grid integer of -x is -x'); with add_q non-null the kernel also
// writes sum_q = add_q + these residues, reduced to the balanced range
// (the residues of the sum of the two grid integers, e.g. Ar' + Ai').
__global__ void __launch_bounds__(512, 2)
oz_crt_residues(const double* __restrict__ xh, const double* __restrict__ xl, int64_t sr,
                int64_t sl, int64_t rows, int64_t k, const int* __restrict__ exps, int count,
                int p, CrtResidueConsts cst, int8_t* __restrict__ q, int64_t ldq,
                int64_t plane, double sign, const int8_t* __restrict__ add_q,
                int8_t* __restrict__ sum_q) {
  // element l of a staged row sits at column l + l/8 (one padding double
  // every 8), so the 16 threads of a row, reading 8 consecutive elements each,
  // hit distinct banks; the odd row pitch staggers the rows
  constexpr int PITCH = 145;
  __shared__ double t[2][32][PITCH];
  auto col = [](int l) { return l + (l >> 3); };
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * 32;
  const int64_t l0 = (int64_t)blockIdx.x * 128;
  const bool lanes_on_r = (sr == 1);
  {
    // entry e of the block: lanes on r, 32 consecutive rows per half-wave;
    // else 64 consecutive l of one row per wave
    double v[2][8];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const double* __restrict__ src = half ? xl : xh;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int e = tid + 512 * c;             // 0 .. 4095 over the 32 x 128 block
        const int ri = lanes_on_r ? (e & 31) : (e >> 7);
        const int li = lanes_on_r ? (e >> 5) : (e & 127);
        const int64_t rg = r0 + ri, lg = l0 + li;
        v[half][c] = (rg < rows && lg < k) ? src[rg * sr + lg * sl] : 0.0;
      }
    }
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int e = tid + 512 * c;
        const int ri = lanes_on_r ? (e & 31) : (e >> 7);
        const int li = lanes_on_r ? (e >> 5) : (e & 127);
        t[half][ri][col(li)] = v[half][c];
      }
  }
  __syncthreads();
  const int row = tid >> 4, lq = (tid & 15) * 8;
  if (l0 + lq >= ldq) return;
  const int sh = p - ((r0 + row < rows) ? exps[r0 + row] : 0);
  double u1[8], u0[8], w1[8], w0[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int c = col(lq) + i;                 // lq is a multiple of 8
    const double zh = ldexp(sign * t[0][row][c], sh), zl = ldexp(sign * t[1][row][c], sh);
    const double t1 = rint(zh);
    const double t2 = rint((zh - t1) + zl);
    const double u = rint(t1 * 0x1p-52);
    const double w = fma(-u, 0x1p52, t1) + t2;
    u1[i] = rint(u * 0x1p-26);
    u0[i] = fma(-u1[i], 0x1p26, u);
    w1[i] = rint(w * 0x1p-26);
    w0[i] = fma(-w1[i], 0x1p26, w);
  }
  const int64_t off = (r0 + row) * ldq + l0 + lq;
  int8_t* o = q + off;
  // residues of the sum: byte-wise add, then one correction into the
  // balanced range (|a + b| <= m - 1 for odd m; modulo 256 the byte add wraps)
  auto add_store = [&](int m, const uint32_t (&word)[2]) {
    const uint2 a = *(const uint2*)(add_q + (int64_t)m * plane + off);
    const int mm = (int)cst.m[m], h = (mm - 1) / 2;
    uint32_t out[2] = {0u, 0u};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t aw = (i < 4) ? a.x : a.y;
      int v = (int)(int8_t)(aw >> (8 * (i & 3))) + (int)(int8_t)(word[i >> 2] >> (8 * (i & 3)));
      if (m > 0) v = (v > h) ? v - mm : (v < -h) ? v + mm : v;
      out[i >> 2] |= ((uint32_t)v & 0xFFu) << (8 * (i & 3));
    }
    *(uint2*)(sum_q + (int64_t)m * plane + off) = uint2{out[0], out[1]};
  };
  {
    uint32_t word[2] = {0u, 0u};
#pragma unroll
    for (int i = 0; i < 8; ++i) word[i >> 2] |= ((uint32_t)(int)w0[i] & 0xFFu) << (8 * (i & 3));
    *(uint2*)o = uint2{word[0], word[1]};
    if (add_q) add_store(0, word);
  }
#pragma unroll
  for (int m = 1; m < CRT_MAX_MODULI; ++m) {
    if (m >= count) break;
    uint32_t word[2] = {0u, 0u};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double y =
          fma(u1[i], cst.c78[m], fma(u0[i], cst.c52[m], fma(w1[i], cst.c26[m], w0[i])));
      const double qq = rint(y * cst.minv[m]);
      const double r = fma(-qq, cst.m[m], y);
      word[i >> 2] |= ((uint32_t)(int)r & 0xFFu) << (8 * (i & 3));
    }
    *(uint2*)(o + (int64_t)m * plane) = uint2{word[0], word[1]};
    if (add_q) add_store(m, word);
  }
}

// The exact integer X = S - q M from its limb sums S_l (S = sum_l S_l 2^(39 l)
// congruent to X modulo M, |S_l| < 2^51, |X| <= M/4), rounded to a dd: q =
// rint(sum_l S_l g_l), X_l = S_l - q M_l (exact), carries into balanced limbs,
// then DWPlusFP from the lowest limb up.
template <int L>
__device__ __forceinline__ ddv crt_limbs_to_dd(const double (&s)[L], const CrtCombineConsts& cst) {
  double est = 0.0;
#pragma unroll
  for (int l = L - 1; l >= 0; --l) est = fma(s[l], cst.g[l], est);
  const double qm = rint(est);
  double xl[L];
#pragma unroll
  for (int l = 0; l < L; ++l) xl[l] = fma(-qm, cst.ml[l], s[l]);
#pragma unroll
  for (int l = 0; l + 1 < L; ++l) {
    const double c = rint(xl[l] * 0x1p-39);
    xl[l] = fma(-c, 0x1p39, xl[l]);
    xl[l + 1] += c;
  }
  ddv acc{xl[0], 0.0};
#pragma unroll
  for (int l = 1; l < L; ++l) acc = dd_add_d(acc, ldexp(xl[l], CRT_LIMB_BITS * l));
  return acc;
}

// Reconstruction: entry (i, j) from the balanced residues r_t of its
// `count` per-modulus products (int8 planes, entry at plane t, [j*mp + i]).
// S = sum_t r_t W_t is congruent to the product X modulo M, and
// |S| <= 32 * 128 * M; it is accumulated exactly in L limbs of 39 bits
// (S_l = sum_t r_t W_t,l, |S_l| < 2^51, exact in binary64).  q = rint(S / M)
// (estimated as sum_l S_l g_l, error far below the 1/4 margin: |X| <= M/4)
// is removed limb by limb (|q M_l| < 2^51: exact), which leaves the exact
// integer product X = S - q M in limbs; carries bring every limb but the top
// one into [-2^38, 2^38] (each step exact), and the limbs are added into a
// dd from the lowest up (DWPlusFP: relative error about 2^-104 overall).
// Finally X 2^(sigma_i + tau_j - 2P) and C = alpha X' + beta C, as in
// oz_combine.  Four consecutive rows per thread (one 4-byte load per
// modulus); a triangle (tri 1 upper, 2 lower) updates only its entries.
template <int L>
__global__ void __launch_bounds__(256)
oz_crt_combine(const int8_t* __restrict__ x, int64_t mp, int64_t np, int count, int p,
               CrtCombineConsts cst, const int* __restrict__ ea, const int* __restrict__ eb,
               int64_t m, int64_t n, double alpha_hi, double alpha_lo, double beta_hi,
               double beta_lo, int beta_zero, double* __restrict__ c_hi,
               double* __restrict__ c_lo, int64_t ldc, int tri) {
  constexpr int NB = 8;
  const int64_t mq = (m + 3) / 4;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= mq * n) return;
  const int64_t i0 = (gid % mq) * 4, j = gid / mq;
  const int64_t ilo = (tri == 2) ? j : 0, ihi = (tri == 1) ? j : m - 1;
  if (i0 > ihi || i0 + 3 < ilo) return;
  auto updated = [&](int64_t i) { return i < m && i >= ilo && i <= ihi; };
  const int8_t* xp = x + j * mp + i0;
  const int64_t plane = mp * np;
  double ch[4] = {0.0, 0.0, 0.0, 0.0}, cl[4] = {0.0, 0.0, 0.0, 0.0};
  if (!beta_zero) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (updated(i0 + r)) {
        ch[r] = c_hi[i0 + r + j * ldc];
        cl[r] = c_lo[i0 + r + j * ldc];
      }
  }
  double s[4][L];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int l = 0; l < L; ++l) s[r][l] = 0.0;
#pragma unroll
  for (int t0 = 0; t0 < CRT_MAX_MODULI; t0 += NB) {
    if (t0 >= count) break;
    uint32_t v[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u)
      v[u] = (t0 + u < count) ? *(const uint32_t*)(xp + (int64_t)(t0 + u) * plane) : 0u;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int tt = t0 + u;
      if (tt >= count) break;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double res = (double)(int)(int8_t)(v[u] >> (8 * r));
#pragma unroll
        for (int l = 0; l < L; ++l) s[r][l] = fma(res, cst.w[tt][l], s[r][l]);
      }
    }
  }
  const ddv alpha{alpha_hi, alpha_lo}, beta{beta_hi, beta_lo};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t i = i0 + r;
    if (!updated(i)) continue;
    const ddv acc = crt_limbs_to_dd<L>(s[r], cst);
    const int e = ea[i] + eb[j] - 2 * p;
    ddv pr{ldexp(acc.hi, e), ldexp(acc.lo, e)};
    ddv res = dd_mul(alpha, pr);
    const int64_t ci = i + j * ldc;
    if (!beta_zero) res = dd_add(res, dd_mul(beta, ddv{ch[r], cl[r]}));
    c_hi[ci] = res.hi;
    c_lo[ci] = res.lo;
  }
}

// Complex reconstruction: plane t, count + t and 2 count + t hold the
// residues of T1 = Ar' Br', T2 = Ai' Bi' and T3 = (Ar' + Ai')(Br' + Bi')
// modulo modulus t; Re X = T1 - T2 and Im X = T3 - T1 - T2 modulo it
// (|.| <= 384 before the reduction, which rint(y (1/m)) m makes balanced
// exactly), each part rebuilt as in oz_crt_combine and scaled by
// 2^(sigma_i + tau_j - 2P) into the dd planes of P (leading dimension ldp);
// the complex alpha / beta update is the caller's.  Four rows per thread.
template <int L>
__global__ void __launch_bounds__(256)
oz_crt_combine_c(const int8_t* __restrict__ x, int64_t mp, int64_t np, int count, int p,
                 CrtCombineConsts cst, CrtModuli cm, const int* __restrict__ ea,
                 const int* __restrict__ eb, int64_t m, int64_t n, double* __restrict__ prh,
                 double* __restrict__ prl, double* __restrict__ pih, double* __restrict__ pil,
                 int64_t ldp) {
  constexpr int NB = 4;
  const int64_t mq = (m + 3) / 4;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= mq * n) return;
  const int64_t i0 = (gid % mq) * 4, j = gid / mq;
  const int64_t plane = mp * np;
  const int8_t* xp = x + j * mp + i0;
  double sr[4][L], si[4][L];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int l = 0; l < L; ++l) sr[r][l] = si[r][l] = 0.0;
#pragma unroll
  for (int t0 = 0; t0 < CRT_MAX_MODULI; t0 += NB) {
    if (t0 >= count) break;
    uint32_t v1[NB], v2[NB], v3[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const bool on = t0 + u < count;
      const int8_t* q = xp + (int64_t)(t0 + u) * plane;
      v1[u] = on ? *(const uint32_t*)q : 0u;
      v2[u] = on ? *(const uint32_t*)(q + (int64_t)count * plane) : 0u;
      v3[u] = on ? *(const uint32_t*)(q + (int64_t)2 * count * plane) : 0u;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int tt = t0 + u;
      if (tt >= count) break;
      const double mm = cm.m[tt], mi = cm.minv[tt];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a1 = (int)(int8_t)(v1[u] >> (8 * r));
        const int a2 = (int)(int8_t)(v2[u] >> (8 * r));
        const int a3 = (int)(int8_t)(v3[u] >> (8 * r));
        const double yr = (double)(a1 - a2), yi = (double)(a3 - a1 - a2);
        const double re = fma(-rint(yr * mi), mm, yr), im = fma(-rint(yi * mi), mm, yi);
#pragma unroll
        for (int l = 0; l < L; ++l) {
          sr[r][l] = fma(re, cst.w[tt][l], sr[r][l]);
          si[r][l] = fma(im, cst.w[tt][l], si[r][l]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t i = i0 + r;
    if (i >= m) continue;
    const int e = ea[i] + eb[j] - 2 * p;
    const ddv xr = crt_limbs_to_dd<L>(sr[r], cst), xi = crt_limbs_to_dd<L>(si[r], cst);
    const int64_t pi = i + j * ldp;
    prh[pi] = ldexp(xr.hi, e);
    prl[pi] = ldexp(xr.lo, e);
    pih[pi] = ldexp(xi.hi, e);
    pil[pi] = ldexp(xi.lo, e);
  }
}

// qd row operand: residues of X1, X0 and X1 + X0, where X' = X1 2^104 + X0
// is the entry's integer on the grid of 208 bits below 2^sigma_r: each part
// x_p gives t_p = rint(x_p 2^(208 - sigma_r)) (exact scaling), cut into 26-bit
// chunks from the top (j = 7 .. 1: c = rint(t 2^(-26 j)), t -= c 2^(26 j),
// exact; the rest is chunk 0); C_j = sum_p c_pj (|C_j| < 2^28), X0 = sum_{j<4}
// C_j 2^(26 j), X1 = sum_{j>=4} C_j 2^(26 (j-4)).  Per modulus
// y1 = C4 + C5 c26 + C6 c52 + C7 c78 and y0 likewise (< 2^38, exact), each
// reduced as in oz_crt_residues, and the balanced sum of the two residues.
// Planes: X1 residues at q1, X0 at q0, the sums at qs (each count planes of
// rows_p x ldq).  Two of the four parts are staged in LDS at a time
// (37 KB, so the registers, not the LDS, bound the workgroups per CU); a
// thread converts 4 consecutive l of one row (block: 32 rows x
// 64 l) and stores one 4-byte word per modulus and set.
__global__ void __launch_bounds__(512, 2)
oz_crt_residues_qd(const double* __restrict__ x0, const double* __restrict__ x1,
                   const double* __restrict__ x2, const double* __restrict__ x3, int64_t sr,
                   int64_t sl, int64_t rows, int64_t k, const int* __restrict__ exps, int count,
                   CrtResidueConsts cst, int8_t* __restrict__ q1, int8_t* __restrict__ q0,
                   int8_t* __restrict__ qs, int64_t ldq, int64_t plane) {
  constexpr int PITCH = 73;                    // 64 columns + one pad per 8
  __shared__ double t[2][32][PITCH];
  auto col = [](int l) { return l + (l >> 3); };
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * 32;
  const int64_t l0 = (int64_t)blockIdx.x * 64;
  const bool lanes_on_r = (sr == 1);
  const int row = tid >> 4, lq = (tid & 15) * 4;
  const int sh = CRT_QD_GRID_BITS - ((r0 + row < rows) ? exps[r0 + row] : 0);
  double C[8][4];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) C[j][i] = 0.0;
#pragma unroll
  for (int pair = 0; pair < 2; ++pair) {
    if (pair) __syncthreads();                 // the first pair has been read
    double v[2][4];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const double* __restrict__ src = pair ? (half ? x3 : x2) : (half ? x1 : x0);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = tid + 512 * c;           // 0 .. 2047 over the 32 x 64 block
        const int ri = lanes_on_r ? (e & 31) : (e >> 6);
        const int li = lanes_on_r ? (e >> 5) : (e & 63);
        const int64_t rg = r0 + ri, lg = l0 + li;
        v[half][c] = (rg < rows && lg < k) ? src[rg * sr + lg * sl] : 0.0;
      }
    }
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = tid + 512 * c;
        const int ri = lanes_on_r ? (e & 31) : (e >> 6);
        const int li = lanes_on_r ? (e >> 5) : (e & 63);
        t[half][ri][col(li)] = v[half][c];
      }
    __syncthreads();
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double tv = rint(ldexp(t[half][row][col(lq) + i], sh));
#pragma unroll
        for (int j = 7; j >= 1; --j) {
          const double c = rint(ldexp(tv, -26 * j));
          tv = fma(-c, ldexp(1.0, 26 * j), tv);
          C[j][i] += c;
        }
        C[0][i] += tv;
      }
  }
  if (l0 + lq >= ldq) return;
  const int64_t off = (r0 + row) * ldq + l0 + lq;
#pragma unroll
  for (int m = 0; m < CRT_MAX_MODULI; ++m) {
    if (m >= count) break;
    const double mm = cst.m[m], mi = cst.minv[m];
    const int mint = (int)mm, h = (mint - 1) / 2;
    uint32_t w1 = 0u, w0 = 0u, ws = 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double y1 = fma(C[7][i], cst.c78[m], fma(C[6][i], cst.c52[m],
                                                      fma(C[5][i], cst.c26[m], C[4][i])));
      const double y0 = fma(C[3][i], cst.c78[m], fma(C[2][i], cst.c52[m],
                                                      fma(C[1][i], cst.c26[m], C[0][i])));
      const int a = (int)fma(-rint(y1 * mi), mm, y1), b = (int)fma(-rint(y0 * mi), mm, y0);
      int sum = a + b;
      if (m > 0) sum = (sum > h) ? sum - mint : (sum < -h) ? sum + mint : sum;
      w1 |= ((uint32_t)a & 0xFFu) << (8 * i);
      w0 |= ((uint32_t)b & 0xFFu) << (8 * i);
      ws |= ((uint32_t)sum & 0xFFu) << (8 * i);
    }
    *(uint32_t*)(q1 + (int64_t)m * plane + off) = w1;
    *(uint32_t*)(q0 + (int64_t)m * plane + off) = w0;
    *(uint32_t*)(qs + (int64_t)m * plane + off) = ws;
  }
}

// qd reconstruction, one entry per thread: the residues of A = X1 Y1 (planes
// 0 .. count-1), B = X0 Y0 (count ..) and C = (X1 + X0)(Y1 + Y0) (2 count ..)
// give each of the three exactly in 26-bit limbs, as in crt_limbs_to_dd
// (|S_l| < 2^39; q M_l < 2^39), with carries into balanced limbs; then the
// product A 2^208 + (C - A - B) 2^104 + B limb by limb (offsets 8 and 4
// limbs), carried again, and the limbs, scaled by 2^(26 l + sigma_i + tau_j
// - 416), added into a qd from the lowest up, two limbs at a time (TwoSum
// cascade and renormalisation per pair); then C = alpha P + beta C in qd as
// oz_combine_qd.
__global__ void __launch_bounds__(256)
oz_crt_combine_qdm(const int8_t* __restrict__ x, int64_t mp, int64_t np, int count,
                   CrtCombineConsts26 cst, const int* __restrict__ ea,
                   const int* __restrict__ eb, int64_t m, int64_t n, double4 alpha, double4 beta,
                   int beta_zero, double* __restrict__ c0, double* __restrict__ c1,
                   double* __restrict__ c2, double* __restrict__ c3, int64_t ldc) {
  constexpr int L = CRT_MAX_LIMBS26;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= m * n) return;
  const int64_t i = gid % m, j = gid / m;
  const int64_t plane = mp * np;
  const int8_t* xp = x + j * mp + i;
  double sa[L], sb[L], sc[L];
#pragma unroll
  for (int l = 0; l < L; ++l) sa[l] = sb[l] = sc[l] = 0.0;
#pragma unroll
  for (int t = 0; t < CRT_MAX_MODULI; ++t) {
    if (t >= count) break;
    const double ra = (double)xp[(int64_t)t * plane];
    const double rb = (double)xp[(int64_t)(count + t) * plane];
    const double rc = (double)xp[(int64_t)(2 * count + t) * plane];
#pragma unroll
    for (int l = 0; l < L; ++l) {
      sa[l] = fma(ra, cst.w[t][l], sa[l]);
      sb[l] = fma(rb, cst.w[t][l], sb[l]);
      sc[l] = fma(rc, cst.w[t][l], sc[l]);
    }
  }
  // each sum minus its multiple of M, exact limbs
  auto finish = [&](double (&s)[L]) {
    double est = 0.0;
#pragma unroll
    for (int l = L - 1; l >= 0; --l) est = fma(s[l], cst.g[l], est);
    const double qm = rint(est);
#pragma unroll
    for (int l = 0; l < L; ++l) s[l] = fma(-qm, cst.ml[l], s[l]);
  };
  finish(sa);
  finish(sb);
  finish(sc);
  // P = A 2^208 + (C - A - B) 2^104 + B in limbs of 26 bits
  constexpr int T = L + 8;
  double tl[T];
#pragma unroll
  for (int l = 0; l < T; ++l) tl[l] = 0.0;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    tl[l] += sb[l];
    tl[l + 4] += sc[l] - sa[l] - sb[l];
    tl[l + 8] += sa[l];
  }
#pragma unroll
  for (int l = 0; l + 1 < T; ++l) {
    const double c = rint(tl[l] * 0x1p-26);
    tl[l] = fma(-c, 0x1p26, tl[l]);
    tl[l + 1] += c;
  }
  // two balanced limbs make one exact binary64 (|l0 + l1 2^26| < 2^52), so
  // the qd takes T / 2 additions
  const int e = ea[i] + eb[j] - 2 * CRT_QD_GRID_BITS;
  qacc p{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int l = 0; l < T; l += 2) {
    const double pair = fma(tl[l + 1], 0x1p26, tl[l]);
    const double v = ldexp(pair, 26 * l + e);
    double er;
    ts(p.s0, v, p.s0, er);
    ts(p.s1, er, p.s1, er);
    ts(p.s2, er, p.s2, er);
    p.s3 = p.s3 + er;
    qd_renorm(p);
  }
  const double4 ps = qd_final(p);
  const int64_t ci = i + j * ldc;
  qacc r{0.0, 0.0, 0.0, 0.0};
  qd_madd(r, alpha, ps);
  if (!beta_zero) {
    qd_renorm(r);
    qd_madd(r, beta, double4{c0[ci], c1[ci], c2[ci], c3[ci]});
  }
  const double4 o = qd_final(r);
  c0[ci] = o.x;
  c1[ci] = o.y;
  c2[ci] = o.z;
  c3[ci] = o.w;
}

// ---- host orchestration -------------------------------------------------------------

static int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Digit widths of a kind for k terms and nslices slices.
static bool digit_widths(int algo, int64_t k, int nslices, int& wfirst, int& w) {
  if (algo == MPDD_OZAKI_I8) {
    // |X_d| <= nslices * k * 2^(2w-2) must stay below 2^31: 8-bit later
    // digits (|q| <= 128) while nslices * k < 2^17, 7-bit ones (|q| <= 64)
    // while nslices * k < 2^19
    const int64_t terms = (int64_t)nslices * k;
    wfirst = 6;
    w = (terms < ((int64_t)1 << 17)) ? 8 : 7;
    return terms < ((int64_t)1 << 19);
  }
  int64_t terms = std::max<int64_t>(1, (int64_t)nslices * k);
  int lg = 0;
  while (((int64_t)1 << lg) < terms) ++lg;
  w = (55 - lg) / 2;
  wfirst = w - 1;
  return wfirst >= 1;
}

// Scale exponents + slices of one row operand (rows x k) into padded buffers.
// `part` is scratch for the chunked maxima (rows * ceil(k / OZ_SCALE_CHUNK)
// doubles, only used when the rows are contiguous across lanes).
// Scale exponents of one row operand (rows x k) from its leading plane.
// hi2 (may be null): a second plane of the same layout whose entries count
// as well (one exponent for the real and imaginary parts of a complex row).
static void scale_operand(const double* hi, int64_t sr, int64_t sl, int64_t rows, int64_t k,
                          int* exps, double* part, hipStream_t st, const double* hi2 = nullptr) {
  if (sl == 1 || k == 0) {
    hipLaunchKernelGGL(oz_scale_rows_wave, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st,
                       hi, hi2, sr, sl, rows, k, exps);
  } else {
    const int nchunks = (int)((k + OZ_SCALE_CHUNK - 1) / OZ_SCALE_CHUNK);
    hipLaunchKernelGGL(oz_scale_part_cols, dim3((unsigned)((rows + 63) / 64), nchunks), dim3(256),
                       0, st, hi, hi2, sr, sl, rows, k, part);
    hipLaunchKernelGGL(oz_scale_finish, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st,
                       part, rows, nchunks, exps);
  }
}

template <typename T>
static hipError_t split_operand(const double* hi, const double* lo, int64_t sr, int64_t sl,
                                int64_t rows, int64_t k, int* exps, T* q, int64_t ldq,
                                int64_t rows_p, int nslices, int wfirst, int w, double* part,
                                hipStream_t st) {
  scale_operand(hi, sr, sl, rows, k, exps, part, st);
  dim3 grid((unsigned)(ldq / 64), (unsigned)(rows_p / 64));
  hipLaunchKernelGGL(oz_slice<T>, grid, dim3(512), 0, st, hi, lo, sr, sl, rows, k, exps, nslices,
                     wfirst, w, q, ldq, rows_p * ldq);
  return hipGetLastError();
}

static size_t part_bytes(int64_t rows, int64_t k) {
  const int64_t nchunks = (k + OZ_SCALE_CHUNK - 1) / OZ_SCALE_CHUNK;
  return (size_t)((rows * std::max<int64_t>(nchunks, 1) * 8 + 255) / 256 * 256);
}

// Workgroup tile (rows, columns) of an INT8 product variant.
static int i8_tile_rows(int var) { return var == 2 ? 128 : 256; }
static int i8_tile_cols(int var) { return (var == 0 || var >= 3) ? 256 : 128; }

// One launch of the INT8 slice products of every anti-diagonal (variant var).
static void launch_i8_products(int var, unsigned nblocks, const int8_t* qa, const int8_t* qb,
                               int32_t* x, int64_t kp, int64_t mp, int64_t np, int s, int tiles_m,
                               int tiles_n, int tri, hipStream_t st) {
  if (var >= 5) {
    auto kern = (var == 5)   ? oz_gemm_i8_dma<256, 256, 2, 4, 4, false, false>
                : (var == 6) ? oz_gemm_i8_dma<256, 256, 2, 4, 4, true, false>
                : (var == 7) ? oz_gemm_i8_dma<256, 256, 2, 2, 4, true, false>
                             : oz_gemm_i8_dma<256, 256, 2, 4, 4, true, true>;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(var == 7 ? 256 : 512), 0, st, qa, qb, x, kp,
                       mp * kp, np * kp, mp, np, s, tiles_m, tiles_n, tri, CrtModuli{}, 1, 0, 1);
    return;
  }
  auto kern = (var == 0)   ? oz_gemm_i8<256, 256, 2, 2>
              : (var == 1) ? oz_gemm_i8<256, 128, 2, 2>
              : (var == 2) ? oz_gemm_i8<128, 128, 2, 2>
              : (var == 3) ? oz_gemm_i8<256, 256, 2, 4>
                           : oz_gemm_i8<256, 256, 4, 4>;
  const unsigned nthreads = (var == 4) ? 1024 : (var >= 3) ? 512 : 256;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(nthreads), 0, st, qa, qb, x, kp, mp * kp, np * kp,
                     mp, np, s, tiles_m, tiles_n, tri);
}

// The residue products of the modular form: one group of workgroups per
// modulus, entries reduced to int8 residues (variants 5, 6 and 8; 6 is the
// default).
static bool crt_variant(int var) { return var == 5 || var == 6 || var == 8; }

// nprod products of residue planes (plane t of both operands into plane t
// of x), plane t modulo modulus t % count.  A workgroup takes a group of
// consecutive planes of its tile when the k-sweep is short (k <= 4096: 2,
// k <= 2048: 4), so that the pipeline fill and drain are paid once per
// group.
static void launch_crt_products(int var, const int8_t* qa, const int8_t* qb, int8_t* x,
                                int64_t kp, int64_t mp, int64_t np, int nprod, int count,
                                int tiles_m, int tiles_n, int tri, const CrtModuli& cm,
                                hipStream_t st) {
  auto kern = (var == 5)   ? oz_gemm_i8_dma<256, 256, 2, 4, 4, false, false, true>
              : (var == 6) ? oz_gemm_i8_dma<256, 256, 2, 4, 4, true, false, true>
                           : oz_gemm_i8_dma<256, 256, 2, 4, 4, true, true, true>;
  const int64_t ksteps = kp / I8_BK;
  const int group = (ksteps <= 32) ? 4 : (ksteps <= 64) ? 2 : 1;
  const int ngroups = (nprod + group - 1) / group;
  const unsigned nblocks = (unsigned)(oz_group_tiles(tri, tiles_m, tiles_n) * ngroups);
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(512), 0, st, qa, qb, (int32_t*)x, kp, mp * kp,
                     np * kp, mp, np, ngroups, tiles_m, tiles_n, tri, cm, count, nprod, group);
}

// Residues of one row operand (scale exponents first).
static void launch_crt_residues(const double* hi, const double* lo, int64_t sr, int64_t sl,
                                int64_t rows, int64_t k, const int* exps, int8_t* q, int64_t ldq,
                                int64_t rows_p, int count, int p, const CrtResidueConsts& rc,
                                hipStream_t st, double sign = 1.0,
                                const int8_t* add_q = nullptr, int8_t* sum_q = nullptr) {
  dim3 grid((unsigned)((ldq + 127) / 128), (unsigned)(rows_p / 32));
  hipLaunchKernelGGL(oz_crt_residues, grid, dim3(512), 0, st, hi, lo, sr, sl, rows, k, exps,
                     count, p, rc, q, ldq, rows_p * ldq, sign, add_q, sum_q);
}

static hipError_t crt_operand(const double* hi, const double* lo, int64_t sr, int64_t sl,
                              int64_t rows, int64_t k, int* exps, int8_t* q, int64_t ldq,
                              int64_t rows_p, int count, int p, const CrtResidueConsts& rc,
                              double* part, hipStream_t st) {
  scale_operand(hi, sr, sl, rows, k, exps, part, st);
  launch_crt_residues(hi, lo, sr, sl, rows, k, exps, q, ldq, rows_p, count, p, rc, st);
  return hipGetLastError();
}

static void launch_crt_combine(int limbs, const int8_t* x, int64_t mp, int64_t np, int count,
                               int p, const CrtCombineConsts& cc, const int* ea, const int* eb,
                               int64_t m, int64_t n, double alpha_hi, double alpha_lo,
                               double beta_hi, double beta_lo, int beta_zero, double* c_hi,
                               double* c_lo, int64_t ldc, int tri, hipStream_t st) {
  auto kern = (limbs <= 1)   ? oz_crt_combine<1>
              : (limbs == 2) ? oz_crt_combine<2>
              : (limbs == 3) ? oz_crt_combine<3>
              : (limbs == 4) ? oz_crt_combine<4>
              : (limbs == 5) ? oz_crt_combine<5>
              : (limbs == 6) ? oz_crt_combine<6>
                             : oz_crt_combine<7>;
  const unsigned cb = (unsigned)(((m + 3) / 4 * n + 255) / 256);
  hipLaunchKernelGGL(kern, dim3(cb), dim3(256), 0, st, x, mp, np, count, p, cc, ea, eb, m, n,
                     alpha_hi, alpha_lo, beta_hi, beta_lo, beta_zero, c_hi, c_lo, ldc, tri);
}

// Modular split form (MPDD_OZAKI_CRT): residues of op(A) and op(B) (a
// triangle: op(A)'s serve both), one INT8 product per modulus, reconstruction.
// alpha = 0 and k = 0 are the caller's.
static int ozaki_crt_gemm(const mpdd_opts* opts, int tri, bool ta, bool tb, int64_t m,
                          int64_t n, int64_t k, double alpha_hi, double alpha_lo,
                          const double* a_hi, const double* a_lo, int64_t lda,
                          const double* b_hi, const double* b_lo, int64_t ldb, double beta_hi,
                          double beta_lo, double* c_hi, double* c_lo, int64_t ldc,
                          hipStream_t st, hipMemPool_t pool) {
  const int count = opts->nslices ? opts->nslices : crt_default_count(k);
  if (count < 1 || count > CRT_MAX_MODULI || k > CRT_MAX_K) return MPDD_ERR_UNSUPPORTED;
  const int p = crt_exponent(k, count);
  if (p == 0) return MPDD_ERR_UNSUPPORTED;
  const int var = opts->tile_id >= 0 ? opts->tile_id : 6;
  if (!crt_variant(var)) return MPDD_ERR_UNSUPPORTED;
  CrtResidueConsts rc;
  CrtModuli cm;
  CrtCombineConsts cc;
  const int limbs = crt_constants(count, &rc, &cm, &cc);
  const bool beta_zero = beta_hi == 0.0 && beta_lo == 0.0;
  const int64_t kp = round_up(k, 2 * I8_BK);
  const int64_t mp = round_up(m, I8_PAD), np = round_up(n, I8_PAD);
  const size_t qa_bytes = (size_t)count * mp * kp;
  const size_t qb_bytes = tri ? 0 : (size_t)count * np * kp;
  const size_t x_bytes = (size_t)count * mp * np;   // int8 residues of the products
  const size_t e_bytes = round_up((m + n) * sizeof(int), 256);
  const size_t p_bytes = std::max(part_bytes(m, k), part_bytes(n, k));
  void* ws = nullptr;
  if (hipMallocFromPoolAsync(&ws, round_up(qa_bytes, 256) + round_up(qb_bytes, 256) + x_bytes +
                                      e_bytes + p_bytes,
                             pool, st) != hipSuccess)
    return MPDD_ERR_ALLOC;
  int8_t* qa = (int8_t*)ws;
  int8_t* qb = tri ? qa : qa + round_up(qa_bytes, 256);
  int8_t* x = (int8_t*)ws + round_up(qa_bytes, 256) + round_up(qb_bytes, 256);
  int* ea = (int*)((char*)x + x_bytes);
  int* eb = tri ? ea : ea + m;
  double* part = (double*)((char*)ea + e_bytes);
  const int64_t a_sr = ta ? lda : 1, a_sl = ta ? 1 : lda;
  const int64_t b_sr = tb ? 1 : ldb, b_sl = tb ? ldb : 1;
  hipError_t e = crt_operand(a_hi, a_lo, a_sr, a_sl, m, k, ea, qa, kp, mp, count, p, rc, part, st);
  if (e == hipSuccess && !tri)
    e = crt_operand(b_hi, b_lo, b_sr, b_sl, n, k, eb, qb, kp, np, count, p, rc, part, st);
  if (e == hipSuccess) {
    const int tiles_m = (int)(mp / i8_tile_rows(var)), tiles_n = (int)(np / i8_tile_cols(var));
    launch_crt_products(var, qa, qb, x, kp, mp, np, count, count, tiles_m, tiles_n, tri, cm, st);
    launch_crt_combine(limbs, x, mp, np, count, p, cc, ea, eb, m, n, alpha_hi, alpha_lo, beta_hi,
                       beta_lo, (int)beta_zero, c_hi, c_lo, ldc, tri, st);
    e = hipGetLastError();
  }
  const hipError_t ef = hipFreeAsync(ws, st);
  if (e != hipSuccess || ef != hipSuccess) return MPDD_ERR_HIP;
  return 0;
}

int ozaki_crt_cgemm(const void* opts_v, int opa, int opb, int64_t m, int64_t n, int64_t k,
                    const double* const* a, int64_t lda, const double* const* b, int64_t ldb,
                    double* prh, double* prl, double* pih, double* pil, hipStream_t st,
                    hipMemPool_t pool) {
  const mpdd_opts* opts = (const mpdd_opts*)opts_v;
  const int count = opts->nslices ? opts->nslices : crt_default_count(k, 3);
  if (count < 1 || count > CRT_MAX_MODULI || k > CRT_MAX_K) return MPDD_ERR_UNSUPPORTED;
  const int p = crt_exponent(k, count, 3);
  if (p == 0) return MPDD_ERR_UNSUPPORTED;
  const int var = opts->tile_id >= 0 ? opts->tile_id : 6;
  if (!crt_variant(var)) return MPDD_ERR_UNSUPPORTED;
  CrtResidueConsts rc;
  CrtModuli cm;
  CrtCombineConsts cc;
  const int limbs = crt_constants(count, &rc, &cm, &cc);
  const int64_t kp = round_up(k, 2 * I8_BK);
  const int64_t mp = round_up(m, I8_PAD), np = round_up(n, I8_PAD);
  // three residue sets per operand (re, im, re + im) and three products
  const size_t qa_bytes = (size_t)3 * count * mp * kp, qb_bytes = (size_t)3 * count * np * kp;
  const size_t x_bytes = (size_t)3 * count * mp * np;
  const size_t e_bytes = round_up((m + n) * sizeof(int), 256);
  const size_t p_bytes = std::max(part_bytes(m, k), part_bytes(n, k));
  void* ws = nullptr;
  if (hipMallocFromPoolAsync(&ws, round_up(qa_bytes, 256) + round_up(qb_bytes, 256) + x_bytes +
                                      e_bytes + p_bytes,
                             pool, st) != hipSuccess)
    return MPDD_ERR_ALLOC;
  int8_t* qa = (int8_t*)ws;
  int8_t* qb = qa + round_up(qa_bytes, 256);
  int8_t* x = qb + round_up(qb_bytes, 256);
  int* ea = (int*)(x + x_bytes);
  int* eb = ea + m;
  double* part = (double*)((char*)ea + e_bytes);
  const int64_t a_sr = opa ? lda : 1, a_sl = opa ? 1 : lda;
  const int64_t b_sr = opb ? 1 : ldb, b_sl = opb ? ldb : 1;
  const int64_t sa = (int64_t)count * mp * kp, sb = (int64_t)count * np * kp;
  // one exponent per row over both parts; the imaginary residues negated for
  // a conjugated operand, and the residues of re + im formed beside them
  scale_operand(a[0], a_sr, a_sl, m, k, ea, part, st, a[2]);
  launch_crt_residues(a[0], a[1], a_sr, a_sl, m, k, ea, qa, kp, mp, count, p, rc, st);
  launch_crt_residues(a[2], a[3], a_sr, a_sl, m, k, ea, qa + sa, kp, mp, count, p, rc, st,
                      opa == 2 ? -1.0 : 1.0, qa, qa + 2 * sa);
  scale_operand(b[0], b_sr, b_sl, n, k, eb, part, st, b[2]);
  launch_crt_residues(b[0], b[1], b_sr, b_sl, n, k, eb, qb, kp, np, count, p, rc, st);
  launch_crt_residues(b[2], b[3], b_sr, b_sl, n, k, eb, qb + sb, kp, np, count, p, rc, st,
                      opb == 2 ? -1.0 : 1.0, qb, qb + 2 * sb);
  const int tiles_m = (int)(mp / i8_tile_rows(var)), tiles_n = (int)(np / i8_tile_cols(var));
  launch_crt_products(var, qa, qb, x, kp, mp, np, 3 * count, count, tiles_m, tiles_n, 0, cm, st);
  auto kern = (limbs <= 1)   ? oz_crt_combine_c<1>
              : (limbs == 2) ? oz_crt_combine_c<2>
              : (limbs == 3) ? oz_crt_combine_c<3>
              : (limbs == 4) ? oz_crt_combine_c<4>
              : (limbs == 5) ? oz_crt_combine_c<5>
              : (limbs == 6) ? oz_crt_combine_c<6>
                             : oz_crt_combine_c<7>;
  const unsigned cbk = (unsigned)(((m + 3) / 4 * n + 255) / 256);
  hipLaunchKernelGGL(kern, dim3(cbk), dim3(256), 0, st, x, mp, np, count, p, cc, cm, ea, eb, m, n,
                     prh, prl, pih, pil, m);
  const hipError_t e = hipGetLastError();
  const hipError_t ef = hipFreeAsync(ws, st);
  if (e != hipSuccess || ef != hipSuccess) return MPDD_ERR_HIP;
  return 0;
}

int ozaki_crt_qgemm(const void* opts_v, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                    const double* alpha, const double* const* a, int64_t lda,
                    const double* const* b, int64_t ldb, const double* beta, int beta_zero,
                    double* const* c, int64_t ldc, hipStream_t st, hipMemPool_t pool) {
  const mpdd_opts* opts = (const mpdd_opts*)opts_v;
  const int count = opts->nslices ? opts->nslices : crt_qd_default_count(k);
  if (k > CRT_MAX_K || !crt_qd_count_ok(k, count)) return MPDD_ERR_UNSUPPORTED;
  const int var = opts->tile_id >= 0 ? opts->tile_id : 6;
  if (!crt_variant(var)) return MPDD_ERR_UNSUPPORTED;
  CrtResidueConsts rc;
  CrtModuli cm;
  CrtCombineConsts cc;
  crt_constants(count, &rc, &cm, &cc);
  CrtCombineConsts26 c26;
  crt_constants26(count, &c26);
  const int64_t kp = round_up(k, 2 * I8_BK);
  const int64_t mp = round_up(m, I8_PAD), np = round_up(n, I8_PAD);
  const size_t qa_bytes = (size_t)3 * count * mp * kp, qb_bytes = (size_t)3 * count * np * kp;
  const size_t x_bytes = (size_t)3 * count * mp * np;
  const size_t e_bytes = round_up((m + n) * sizeof(int), 256);
  const size_t p_bytes = std::max(part_bytes(m, k), part_bytes(n, k));
  void* ws = nullptr;
  if (hipMallocFromPoolAsync(&ws, round_up(qa_bytes, 256) + round_up(qb_bytes, 256) + x_bytes +
                                      e_bytes + p_bytes,
                             pool, st) != hipSuccess)
    return MPDD_ERR_ALLOC;
  int8_t* qa = (int8_t*)ws;
  int8_t* qb = qa + round_up(qa_bytes, 256);
  int8_t* x = qb + round_up(qb_bytes, 256);
  int* ea = (int*)(x + x_bytes);
  int* eb = ea + m;
  double* part = (double*)((char*)ea + e_bytes);
  const int64_t a_sr = ta ? lda : 1, a_sl = ta ? 1 : lda;
  const int64_t b_sr = tb ? 1 : ldb, b_sl = tb ? ldb : 1;
  const int64_t sa = (int64_t)count * mp * kp, sb = (int64_t)count * np * kp;
  // residue sets: X1 (planes 0 ..), X0 (count ..), X1 + X0 (2 count ..)
  scale_operand(a[0], a_sr, a_sl, m, k, ea, part, st);
  hipLaunchKernelGGL(oz_crt_residues_qd, dim3((unsigned)(kp / 64), (unsigned)(mp / 32)),
                     dim3(512), 0, st, a[0], a[1], a[2], a[3], a_sr, a_sl, m, k, ea, count, rc,
                     qa, qa + sa, qa + 2 * sa, kp, mp * kp);
  scale_operand(b[0], b_sr, b_sl, n, k, eb, part, st);
  hipLaunchKernelGGL(oz_crt_residues_qd, dim3((unsigned)(kp / 64), (unsigned)(np / 32)),
                     dim3(512), 0, st, b[0], b[1], b[2], b[3], b_sr, b_sl, n, k, eb, count, rc,
                     qb, qb + sb, qb + 2 * sb, kp, np * kp);
  const int tiles_m = (int)(mp / i8_tile_rows(var)), tiles_n = (int)(np / i8_tile_cols(var));
  launch_crt_products(var, qa, qb, x, kp, mp, np, 3 * count, count, tiles_m, tiles_n, 0, cm, st);
  hipLaunchKernelGGL(oz_crt_combine_qdm, dim3((unsigned)((m * n + 255) / 256)), dim3(256), 0, st,
                     x, mp, np, count, c26, ea, eb, m, n,
                     double4{alpha[0], alpha[1], alpha[2], alpha[3]},
                     double4{beta[0], beta[1], beta[2], beta[3]}, beta_zero, c[0], c[1], c[2],
                     c[3], ldc);
  const hipError_t e = hipGetLastError();
  const hipError_t ef = hipFreeAsync(ws, st);
  if (e != hipSuccess || ef != hipSuccess) return MPDD_ERR_HIP;
  return 0;
}

int ozaki_gemm(const void* opts_v, int tri, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
               double alpha_hi, double alpha_lo, const double* a_hi, const double* a_lo,
               int64_t lda, const double* b_hi, const double* b_lo, int64_t ldb, double beta_hi,
               double beta_lo, double* c_hi, double* c_lo, int64_t ldc, hipStream_t st,
               hipMemPool_t pool) {
  const mpdd_opts* opts = (const mpdd_opts*)opts_v;
  const int algo = opts->algo;
  const bool beta_zero = beta_hi == 0.0 && beta_lo == 0.0;
  if ((alpha_hi == 0.0 && alpha_lo == 0.0) || k == 0) {
    GemmParams p{};
    p.m = m; p.n = n; p.k = k;
    p.beta_hi = beta_hi; p.beta_lo = beta_lo;
    p.c_hi = c_hi; p.c_lo = c_lo; p.ldc = ldc;
    p.beta_zero = beta_zero;
    p.tri = tri;
    return launch_scale(p, st) == hipSuccess ? 0 : MPDD_ERR_HIP;
  }
  if (algo == MPDD_OZAKI_CRT)
    return ozaki_crt_gemm(opts, tri, ta, tb, m, n, k, alpha_hi, alpha_lo, a_hi, a_lo, lda, b_hi,
                          b_lo, ldb, beta_hi, beta_lo, c_hi, c_lo, ldc, st, pool);
  int s = opts->nslices;
  if (s == 0) s = (algo == MPDD_OZAKI_I8) ? 16 : 7;
  if (s < 1 || s > 40) return MPDD_ERR_UNSUPPORTED;
  int wfirst, w;
  if (!digit_widths(algo, k, s, wfirst, w)) return MPDD_ERR_UNSUPPORTED;

  const bool i8 = (algo == MPDD_OZAKI_I8);
  // INT8 slice rows are padded to an even number of product k-steps
  const int64_t kp = round_up(k, i8 ? 2 * I8_BK : OZ_KPAD);
  // INT8 product variant (tile_id) and its workgroup tile
  // (default 6: 256 x 256 with 8 waves -- the largest tile, so the least data
  // moved per product, two waves per SIMD -- with the digits loaded straight
  // into a four-stage LDS ring and each step's fragments read during the
  // previous step's MFMAs; fastest measured at n = 4096 and 8192)
  const int var = (i8 && opts->tile_id >= 0) ? opts->tile_id : 6;
  if (i8 && var > 8) return MPDD_ERR_UNSUPPORTED;
  // a triangle is walked in square tiles (variant 1's are 256 x 128)
  if (tri && i8 && var == 1) return MPDD_ERR_UNSUPPORTED;
  const int64_t tbm = i8 ? i8_tile_rows(var) : OZ_BM;
  const int64_t tbn = i8 ? i8_tile_cols(var) : OZ_BN;
  const int64_t mp = round_up(m, i8 ? I8_PAD : OZ_BM), np = round_up(n, i8 ? I8_PAD : OZ_BN);
  const size_t esz = i8 ? 1 : 8;
  const size_t xsz = i8 ? 4 : 8;
  // a triangle (Rsyrk: op(B) = op(A)^T, m == n) uses op(A)'s slices and
  // exponents for op(B) as well: the columns of op(B) are the rows of op(A)
  const size_t qa_bytes = (size_t)s * mp * kp * esz;
  const size_t qb_bytes = tri ? 0 : (size_t)s * np * kp * esz;
  const size_t x_bytes = (size_t)s * mp * np * xsz;
  const size_t e_bytes = round_up((m + n) * sizeof(int), 256);
  const size_t p_bytes = std::max(part_bytes(m, k), part_bytes(n, k));
  const size_t total =
      round_up(qa_bytes, 256) + round_up(qb_bytes, 256) + x_bytes + e_bytes + p_bytes;
  void* ws = nullptr;
  if (hipMallocFromPoolAsync(&ws, total, pool, st) != hipSuccess) return MPDD_ERR_ALLOC;
  char* base = (char*)ws;
  void* qa = base;
  void* qb = tri ? qa : base + round_up(qa_bytes, 256);
  void* x = base + round_up(qa_bytes, 256) + round_up(qb_bytes, 256);
  int* ea = (int*)((char*)x + x_bytes);
  int* eb = tri ? ea : ea + m;
  double* part = (double*)((char*)ea + e_bytes);

  // row operand of A: op(A)(i, l); of B: op(B)(l, j) as element (j, l)
  const int64_t a_sr = ta ? lda : 1, a_sl = ta ? 1 : lda;
  const int64_t b_sr = tb ? 1 : ldb, b_sl = tb ? ldb : 1;
  hipError_t e;
  if (i8) {
    e = split_operand<int8_t>(a_hi, a_lo, a_sr, a_sl, m, k, ea, (int8_t*)qa, kp, mp, s, wfirst, w,
                              part, st);
    if (e == hipSuccess && !tri)
      e = split_operand<int8_t>(b_hi, b_lo, b_sr, b_sl, n, k, eb, (int8_t*)qb, kp, np, s, wfirst,
                                w, part, st);
  } else {
    e = split_operand<double>(a_hi, a_lo, a_sr, a_sl, m, k, ea, (double*)qa, kp, mp, s, wfirst, w,
                              part, st);
    if (e == hipSuccess && !tri)
      e = split_operand<double>(b_hi, b_lo, b_sr, b_sl, n, k, eb, (double*)qb, kp, np, s, wfirst,
                                w, part, st);
  }
  const int tiles_m = (int)(mp / tbm), tiles_n = (int)(np / tbn);
  const unsigned nblocks = (unsigned)(oz_group_tiles(tri, tiles_m, tiles_n) * s);
  if (e == hipSuccess) {
    if (i8)
      launch_i8_products(var, nblocks, (const int8_t*)qa, (const int8_t*)qb, (int32_t*)x, kp, mp,
                         np, s, tiles_m, tiles_n, tri, st);
    else
      hipLaunchKernelGGL(oz_gemm_f64, dim3(nblocks), dim3(256), 0, st, (const double*)qa,
                         (const double*)qb, (double*)x, kp, mp * kp, np * kp, mp, np, s, tiles_m,
                         tiles_n, tri);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const unsigned cb = (unsigned)(((m + 3) / 4 * n + 255) / 256);
    if (i8)
      hipLaunchKernelGGL(oz_combine<int32_t>, dim3(cb), dim3(256), 0, st, (const int32_t*)x, mp,
                         np, s, wfirst, w, ea, eb, m, n, alpha_hi, alpha_lo, beta_hi, beta_lo,
                         (int)beta_zero, c_hi, c_lo, ldc, tri);
    else
      hipLaunchKernelGGL(oz_combine<double>, dim3(cb), dim3(256), 0, st, (const double*)x, mp, np,
                         s, wfirst, w, ea, eb, m, n, alpha_hi, alpha_lo, beta_hi, beta_lo,
                         (int)beta_zero, c_hi, c_lo, ldc, tri);
    e = hipGetLastError();
  }
  hipError_t ef = hipFreeAsync(ws, st);
  if (e != hipSuccess) return MPDD_ERR_HIP;
  return ef == hipSuccess ? 0 : MPDD_ERR_HIP;
}

// Split-form qd Rgemm (INT8 slices): scale and slice op(A) and op(B) from
// their quad-double planes, the same exact slice products per anti-diagonal
// as the dd form, combined in qd.  alpha = 0 and k = 0 are the caller's.
int ozaki_qgemm(const void* opts_v, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                const double* alpha, const double* const* a, int64_t lda,
                const double* const* b, int64_t ldb, const double* beta, int beta_zero,
                double* const* c, int64_t ldc, hipStream_t st, hipMemPool_t pool) {
  const mpdd_opts* opts = (const mpdd_opts*)opts_v;
  if (opts->algo != MPDD_OZAKI_I8) return MPDD_ERR_UNSUPPORTED;
  int s = opts->nslices;
  if (s == 0) s = 32;
  if (s < 1 || s > OZ_QD_MAX_SLICES) return MPDD_ERR_UNSUPPORTED;
  int wfirst, w;
  if (!digit_widths(MPDD_OZAKI_I8, k, s, wfirst, w)) return MPDD_ERR_UNSUPPORTED;
  const int var = opts->tile_id >= 0 ? opts->tile_id : 6;
  if (var > 8) return MPDD_ERR_UNSUPPORTED;
  const int64_t kp = round_up(k, 2 * I8_BK);
  const int64_t mp = round_up(m, I8_PAD), np = round_up(n, I8_PAD);
  const size_t qa_bytes = (size_t)s * mp * kp, qb_bytes = (size_t)s * np * kp;
  const size_t x_bytes = (size_t)s * mp * np * sizeof(int32_t);
  const size_t e_bytes = round_up((m + n) * sizeof(int), 256);
  const size_t p_bytes = std::max(part_bytes(m, k), part_bytes(n, k));
  void* ws = nullptr;
  if (hipMallocFromPoolAsync(&ws, round_up(qa_bytes, 256) + round_up(qb_bytes, 256) + x_bytes +
                                      e_bytes + p_bytes,
                             pool, st) != hipSuccess)
    return MPDD_ERR_ALLOC;
  int8_t* qa = (int8_t*)ws;
  int8_t* qb = qa + round_up(qa_bytes, 256);
  int32_t* x = (int32_t*)(qb + round_up(qb_bytes, 256));
  int* ea = (int*)((char*)x + x_bytes);
  int* eb = ea + m;
  double* part = (double*)((char*)ea + e_bytes);
  // row operand of A: op(A)(i, l); of B: op(B)(l, j) as element (j, l)
  const int64_t a_sr = ta ? lda : 1, a_sl = ta ? 1 : lda;
  const int64_t b_sr = tb ? 1 : ldb, b_sl = tb ? ldb : 1;
  scale_operand(a[0], a_sr, a_sl, m, k, ea, part, st);
  hipLaunchKernelGGL(oz_slice_qd, dim3((unsigned)(kp / 64), (unsigned)(mp / 64)), dim3(512), 0,
                     st, a[0], a[1], a[2], a[3], a_sr, a_sl, m, k, ea, s, wfirst, w, qa, kp,
                     mp * kp);
  scale_operand(b[0], b_sr, b_sl, n, k, eb, part, st);
  hipLaunchKernelGGL(oz_slice_qd, dim3((unsigned)(kp / 64), (unsigned)(np / 64)), dim3(512), 0,
                     st, b[0], b[1], b[2], b[3], b_sr, b_sl, n, k, eb, s, wfirst, w, qb, kp,
                     np * kp);
  const int tiles_m = (int)(mp / i8_tile_rows(var)), tiles_n = (int)(np / i8_tile_cols(var));
  launch_i8_products(var, (unsigned)(tiles_m * tiles_n * s), qa, qb, x, kp, mp, np, s, tiles_m,
                     tiles_n, 0, st);
  hipLaunchKernelGGL(oz_combine_qd, dim3((unsigned)((m * n + 255) / 256)), dim3(256), 0, st, x,
                     mp, np, s, wfirst, w, ea, eb, m, n,
                     double4{alpha[0], alpha[1], alpha[2], alpha[3]},
                     double4{beta[0], beta[1], beta[2], beta[3]}, beta_zero, c[0], c[1], c[2],
                     c[3], ldc);
  const hipError_t e = hipGetLastError();
  const hipError_t ef = hipFreeAsync(ws, st);
  if (e != hipSuccess || ef != hipSuccess) return MPDD_ERR_HIP;
  return 0;
}

// Exposed building block: scale exponents and digit slices of op(X).
int ozaki_split_entry(int algo, bool trans, int64_t rows, int64_t k, const double* hi,
                      const double* lo, int64_t ld, int nslices, int wfirst, int w, int* exps,
                      void* slices, int64_t ldq, int64_t rows_p, hipStream_t st,
                      hipMemPool_t pool) {
  const int64_t sr = trans ? ld : 1, sl = trans ? 1 : ld;
  void* part = nullptr;
  if (hipMallocFromPoolAsync(&part, part_bytes(rows, k), pool, st) != hipSuccess)
    return MPDD_ERR_ALLOC;
  hipError_t e;
  if (algo == MPDD_OZAKI_CRT) {
    // residues: nslices moduli, the grid of crt_exponent (checked by the caller)
    CrtResidueConsts rc;
    CrtModuli cm;
    CrtCombineConsts cc;
    crt_constants(nslices, &rc, &cm, &cc);
    e = crt_operand(hi, lo, sr, sl, rows, k, exps, (int8_t*)slices, ldq, rows_p, nslices,
                    crt_exponent(k, nslices), rc, (double*)part, st);
  } else if (algo == MPDD_OZAKI_I8)
    e = split_operand<int8_t>(hi, lo, sr, sl, rows, k, exps, (int8_t*)slices, ldq, rows_p,
                              nslices, wfirst, w, (double*)part, st);
  else
    e = split_operand<double>(hi, lo, sr, sl, rows, k, exps, (double*)slices, ldq, rows_p, nslices,
                              wfirst, w, (double*)part, st);
  hipError_t ef = hipFreeAsync(part, st);
  if (e != hipSuccess) return MPDD_ERR_HIP;
  return ef == hipSuccess ? 0 : MPDD_ERR_HIP;
}

int ozaki_digit_widths(int algo, int64_t k, int nslices, int* wfirst, int* w) {
  int a, b;
  if (!digit_widths(algo, k, nslices, a, b)) return MPDD_ERR_UNSUPPORTED;
  *wfirst = a;
  *w = b;
  return 0;
}

}  // namespace mpdd

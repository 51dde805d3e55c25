// gemm_plain.hip -- plain dd Rgemm / Rsyrk kernels for gfx950.
//
// One workgroup computes a BM x BN tile of C.  Each k-tile of op(A)
// (BM x BK) and op(B) (BK x BN) is read from the hi/lo planes in HBM with
// coalesced 8-byte loads (leading dimensions may be odd, so columns are only
// 8-byte aligned), held in registers while the previous k-tile is being
// consumed, and written to LDS as interleaved double2 {hi, lo} so that one
// ds_read_b128 delivers a whole dd operand.  LDS is double buffered: one
// barrier per k-tile.  Each thread owns an RM x RN block of dd accumulators
// (rows tm + TMX*r, columns tn + TNX*c: consecutive lanes read consecutive
// LDS words, so operand reads are conflict-free) and updates it with the dd
// multiply-accumulate of dd.hpp.
//
// The same kernel serves Rsyrk (manual Table "mpblasroutines"): op(B) is
// op(A)^T read from the same planes, only tiles that meet the uplo triangle
// are launched, and the epilogue masks the diagonal tiles element by element
// so the opposite triangle is never written.
//
// With a k-split (skinny products with too few C tiles to fill 256 CUs),
// blockIdx.z selects a k-range; each slice writes its dd partial sums to a
// scratch buffer and dd_splitk_reduce adds them in a fixed order with
// cross-lane shuffles, then applies alpha / beta.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dd.hpp"
#include "kernels.hpp"

typedef double v4d __attribute__((ext_vector_type(4)));

#pragma clang fp contract(off)

namespace mpdd {

// Decode tile coordinates of workgroup b.  Workgroups are dealt round-robin
// to the 8 XCDs; remapping b so that each XCD receives a contiguous run of
// tiles, and walking that run in 8 x 8 blocks of tiles, makes the ~64
// workgroups an XCD runs at once share 8 row panels of op(A) and 8 column
// panels of op(B) in its L2 (instead of 64 row panels and one column panel).
// A triangle (Rsyrk) with a tile count that is a multiple of 8 is walked in
// the same 8 x 8 blocks, taken over the triangle of blocks, so that each XCD
// receives a near-equal share of the work; the workgroups of the tiles of a
// diagonal block that lie outside the triangle return at once (false).
// Other triangles launch only their tiles, column by column.
__device__ __forceinline__ int tri_col(int t) {
  // largest y with y(y+1)/2 <= t
  int y = (int)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((y + 1) * (y + 2) / 2 <= t) ++y;
  while (y * (y + 1) / 2 > t) --y;
  return y;
}

__device__ __forceinline__ bool tile_coords(const GemmParams& p, int& bi, int& bj) {
  int b = blockIdx.x;
  const int nb = gridDim.x;
  if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
  const bool blocks8 = (p.tiles_m & 7) == 0 && (p.tiles_n & 7) == 0;
  if (p.tri == 0) {
    if (blocks8) {
      const int sb = b >> 6, w = b & 63;
      const int sm = p.tiles_m >> 3;
      bi = (sb % sm) * 8 + (w & 7);
      bj = (sb / sm) * 8 + (w >> 3);
    } else {
      bi = b % p.tiles_m;
      bj = b / p.tiles_m;
    }
    return true;
  }
  if (blocks8) {
    const int sb = b >> 6, w = b & 63;
    const int s8 = p.tiles_m >> 3;
    int sx, sy;
    if ((s8 & 15) == 0) {
      // each XCD's run of blocks: its share of the blocks above the diagonal
      // (taken column by column), then its share of the diagonal blocks
      const int nodd = s8 * (s8 - 1) / 2;
      const int per = (nodd + s8) >> 3, oper = nodd >> 3, dper = s8 >> 3;
      const int x = sb / per, j = sb - x * per;
      if (j < oper) {
        const int t = x * oper + j;
        sy = tri_col(t) + 1;               // block (sx, sy), sx < sy
        sx = t - sy * (sy - 1) / 2;
      } else {
        sx = sy = x * dper + (j - oper);
      }
    } else {
      sy = tri_col(sb);                    // block (sx, sy), sx <= sy
      sx = sb - sy * (sy + 1) / 2;
    }
    if (p.tri == 1) {            // upper: tile row <= tile column
      bi = sx * 8 + (w & 7);
      bj = sy * 8 + (w >> 3);
      return bi <= bj;
    }
    bi = sy * 8 + (w & 7);       // lower: tile row >= tile column
    bj = sx * 8 + (w >> 3);
    return bi >= bj;
  }
  // tiles (x, y) with x <= y, enumerated column by column: t = y(y+1)/2 + x
  const int y = tri_col(b), x = b - y * (y + 1) / 2;
  if (p.tri == 1) { bi = x; bj = y; }
  else { bi = y; bj = x; }
  return true;
}

template <int BM, int BN, int BK>
struct DDTileSmem {
  double2 As[2][BK][BM + 1];
  double2 Bs[2][BK][BN + 1];
};

// Accumulate the BM x BN tile at (i0, j0) of op(A) op(B) over k in
// [kbeg, kend) into this thread's RM x RN block of dd accumulators.
template <int BM, int BN, int BK, int RM, int RN, bool TA, bool TB, bool ACC, bool XM = false>
__device__ __forceinline__ void dd_tile_mainloop(const GemmParams& p, int64_t i0, int64_t j0,
                                                 int64_t kbeg, int64_t kend,
                                                 DDTileSmem<BM, BN, BK>& sm, double (&ch)[RM][RN],
                                                 double (&cl)[RM][RN]) {
  constexpr int TMX = BM / RM;
  constexpr int TNX = BN / RN;
  constexpr int NT = TMX * TNX;
  constexpr int AE = BM * BK / NT;   // A-tile elements staged per thread
  constexpr int BE = BN * BK / NT;
  static_assert(AE * NT == BM * BK && BE * NT == BN * BK, "tile not divisible by threads");
  static_assert(NT % BK == 0, "threads must cover whole k-columns");

  auto& As = sm.As;
  auto& Bs = sm.Bs;
  const int tid = threadIdx.x;
  const int tm = tid % TMX;
  const int tn = tid / TMX;

  // Staging map.  Element e of this thread's share of a tile sits at
  // (mn, kk) inside it.  Lanes walk the direction that is contiguous in
  // memory: for op(A) = A (A[i + l*lda]) and op(B) = B^T (B[j + l*ldb]) that
  // is the row/column index, otherwise it is k.
  auto coord = [&](int e, bool mn_contig, int bmn, int& mn, int& kk) {
    const int x = tid + NT * e;
    if (mn_contig) { mn = x % bmn; kk = x / bmn; } else { kk = x % BK; mn = x / BK; }
  };
  // Element offsets relative to the k-tile start, rows/columns clamped into
  // the matrix: values staged for rows >= m (columns >= n) only reach
  // accumulators that are never stored, so any finite in-bounds value will do.
  int64_t aoff[AE], boff[BE];
  int akk[AE], bkk[BE];
#pragma unroll
  for (int e = 0; e < AE; ++e) {
    int mn, kk;
    coord(e, !TA, BM, mn, kk);
    int64_t gi = i0 + mn;
    gi = gi < p.m ? gi : p.m - 1;
    akk[e] = kk;
    aoff[e] = TA ? (int64_t)kk + gi * p.lda : gi + (int64_t)kk * p.lda;
  }
#pragma unroll
  for (int e = 0; e < BE; ++e) {
    int mn, kk;
    coord(e, TB, BN, mn, kk);
    int64_t gj = j0 + mn;
    gj = gj < p.n ? gj : p.n - 1;
    bkk[e] = kk;
    boff[e] = TB ? gj + (int64_t)kk * p.ldb : (int64_t)kk + gj * p.ldb;
  }
  const int64_t astep = TA ? 1 : p.lda;   // distance between consecutive k
  const int64_t bstep = TB ? p.ldb : 1;

#pragma unroll
  for (int r = 0; r < RM; ++r)
#pragma unroll
    for (int c = 0; c < RN; ++c) { ch[r][c] = 0.0; cl[r][c] = 0.0; }

  double ah_r[AE], al_r[AE], bh_r[BE], bl_r[BE];

  // Load the k-tile starting at k0.  `tail`: zero the terms at k >= kend.
  auto load_tiles = [&](int64_t k0, bool tail) {
    const double* pah = p.a_hi + k0 * astep;
    const double* pal = p.a_lo + k0 * astep;
    const double* pbh = p.b_hi + k0 * bstep;
    const double* pbl = p.b_lo + k0 * bstep;
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      double h = 0.0, l = 0.0;
      if (!tail || k0 + akk[e] < kend) { h = pah[aoff[e]]; l = pal[aoff[e]]; }
      ah_r[e] = h;
      al_r[e] = l;
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      double h = 0.0, l = 0.0;
      if (!tail || k0 + bkk[e] < kend) { h = pbh[boff[e]]; l = pbl[boff[e]]; }
      bh_r[e] = h;
      bl_r[e] = l;
    }
  };

  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      int mn, kk;
      coord(e, !TA, BM, mn, kk);
      As[buf][kk][mn] = make_double2(ah_r[e], al_r[e]);
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      int mn, kk;
      coord(e, TB, BN, mn, kk);
      Bs[buf][kk][mn] = make_double2(bh_r[e], bl_r[e]);
    }
  };

  const int64_t nkt = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
  if (nkt > 0) {
    load_tiles(kbeg, nkt == 1);
    store_tiles(0);
  }
  __syncthreads();

  // XM: the cross terms ah*bl + al*bh of every product go to the FP64 matrix
  // cores (v_mfma_f64_16x16x4_f64, accumulating in X) while the vector units
  // run the 10-op leading-product update.  Wave w owns rows 0..BM-1 and the 16
  // columns tn + 16c of its lanes: MFMA block rb covers rows 16rb..16rb+15 and
  // those columns (column q of the block = local column (q%4) + 16(q/4)).
  constexpr bool XMF = XM && !ACC;
  static_assert(!XMF || (TMX == 16 && TNX == 16 && RN == 4 && NT == 256),
                "matrix-core cross terms need the 16 x 16 thread grid");
  const int lane = tid & 63, wv = tid >> 6;
  const int xr = lane & 15, xk = lane >> 4;
  const int xcol = 4 * wv + (lane & 3) + 16 * ((lane & 15) >> 2);
  v4d X[RM];
#pragma unroll
  for (int r = 0; r < RM; ++r) X[r] = v4d{0.0, 0.0, 0.0, 0.0};

  for (int64_t kt = 0; kt < nkt; ++kt) {
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < nkt;
    if (more) load_tiles(kbeg + (kt + 1) * BK, kt + 2 == nkt);
    if constexpr (XMF) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const double2 xb = Bs[cur][kk + xk][xcol];
#pragma unroll
        for (int rb = 0; rb < RM; ++rb) {
          const double2 xa = As[cur][kk + xk][16 * rb + xr];
          X[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa.x, xb.y, X[rb], 0, 0, 0);
          X[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa.y, xb.x, X[rb], 0, 0, 0);
        }
      }
      double ahs[2][RM], bhs[2][RN];
#pragma unroll
      for (int r = 0; r < RM; ++r) ahs[0][r] = As[cur][0][tm + TMX * r].x;
#pragma unroll
      for (int c = 0; c < RN; ++c) bhs[0][c] = Bs[cur][0][tn + TNX * c].x;
#pragma unroll
      for (int kk = 0; kk < BK; ++kk) {
        const int q = kk & 1;
        if (kk + 1 < BK) {
#pragma unroll
          for (int r = 0; r < RM; ++r) ahs[q ^ 1][r] = As[cur][kk + 1][tm + TMX * r].x;
#pragma unroll
          for (int c = 0; c < RN; ++c) bhs[q ^ 1][c] = Bs[cur][kk + 1][tn + TNX * c].x;
        }
#pragma unroll
        for (int x = 0; x < RM * RN; ++x) {
          const int r = x / RN, c = x % RN;
          madd_lean_hi(ch[r][c], cl[r][c], ahs[q][r], bhs[q][c]);
        }
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
          for (int c = 0; c < RN; ++c) asm volatile("" : "+v"(ch[r][c]), "+v"(cl[r][c]));
        asm volatile("" ::: "memory");
      }
      // renormalise every second k-tile (every 32 terms): |sl| stays ~u|sh|
      if ((kt & 1) || !more) {
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
          for (int c = 0; c < RN; ++c) renorm(ch[r][c], cl[r][c]);
      }
      if (more) store_tiles(cur ^ 1);
      __syncthreads();
      continue;
    }
    // Operands of step kk+1 are read from LDS while step kk computes.
    double2 a[2][RM], b[2][RN];
#pragma unroll
    for (int r = 0; r < RM; ++r) a[0][r] = As[cur][0][tm + TMX * r];
#pragma unroll
    for (int c = 0; c < RN; ++c) b[0][c] = Bs[cur][0][tn + TNX * c];
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      const int q = kk & 1;
      if (kk + 1 < BK) {
#pragma unroll
        for (int r = 0; r < RM; ++r) a[q ^ 1][r] = As[cur][kk + 1][tm + TMX * r];
#pragma unroll
        for (int c = 0; c < RN; ++c) b[q ^ 1][c] = Bs[cur][kk + 1][tn + TNX * c];
      }
#pragma unroll
      for (int x = 0; x < RM * RN; ++x) {
        const int r = x / RN, c = x % RN;
        if (ACC)
          madd_accurate(ch[r][c], cl[r][c], a[q][r].x, a[q][r].y, b[q][c].x, b[q][c].y);
        else
          madd_lean(ch[r][c], cl[r][c], a[q][r].x, a[q][r].y, b[q][c].x, b[q][c].y);
      }
      // Fence: this step's arithmetic completes here and no later LDS read is
      // hoisted above it, so only one step of operands is in flight (without
      // it the compiler issues every LDS read of the k-tile up front and
      // spills).  Emits no instructions.
#pragma unroll
      for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int c = 0; c < RN; ++c) asm volatile("" : "+v"(ch[r][c]), "+v"(cl[r][c]));
      asm volatile("" ::: "memory");
    }
    if (!ACC) {
#pragma unroll
      for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int c = 0; c < RN; ++c) renorm(ch[r][c], cl[r][c]);
    }
    if (more) store_tiles(cur ^ 1);
    __syncthreads();
  }
  if constexpr (XMF) {
    // hand the matrix-core cross terms to the threads that own the entries,
    // through LDS (free after the final barrier of the k-loop)
    double* xs = reinterpret_cast<double*>(&sm.As[0][0][0]) + wv * BM * 16;
#pragma unroll
    for (int rb = 0; rb < RM; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e) xs[(16 * rb + 4 * e + xk) * 16 + xr] = X[rb][e];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
      for (int c = 0; c < RN; ++c) {
        cl[r][c] += xs[(tm + TMX * r) * 16 + (tn - 4 * wv) + 4 * c];
        renorm(ch[r][c], cl[r][c]);
      }
    __syncthreads();
  }
}

// Write this thread's block of the tile at (i0, j0): either the k-split
// partial sums into scratch slice z, or C <- alpha*acc + beta*C on the stored
// entries (masked to the triangle for Rsyrk).
template <int BM, int BN, int RM, int RN, bool PARTIAL>
__device__ __forceinline__ void dd_tile_epilogue(const GemmParams& p, int64_t i0, int64_t j0,
                                                 int z, const double (&ch)[RM][RN],
                                                 const double (&cl)[RM][RN]) {
  constexpr int TMX = BM / RM;
  constexpr int TNX = BN / RN;
  const int tm = threadIdx.x % TMX;
  const int tn = threadIdx.x / TMX;
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int64_t i = i0 + tm + TMX * r;
#pragma unroll
    for (int c = 0; c < RN; ++c) {
      const int64_t j = j0 + tn + TNX * c;
      if (i >= p.m || j >= p.n) continue;
      if (PARTIAL) {
        // k-split partial sum (normalised) into scratch [z][j*m + i]
        const int64_t w = (int64_t)z * p.m * p.n + j * p.m + i;
        p.w_hi[w] = ch[r][c];
        p.w_lo[w] = cl[r][c];
        continue;
      }
      if (p.tri == 1 && i > j) continue;
      if (p.tri == 2 && i < j) continue;
      ddv acc{ch[r][c], cl[r][c]};
      ddv v = dd_mul(ddv{p.alpha_hi, p.alpha_lo}, acc);
      const int64_t ci = i + j * p.ldc;
      if (!p.beta_zero)
        v = dd_add(v, dd_mul(ddv{p.beta_hi, p.beta_lo}, ddv{p.c_hi[ci], p.c_lo[ci]}));
      p.c_hi[ci] = v.hi;
      p.c_lo[ci] = v.lo;
    }
  }
}

template <int BM, int BN, int BK, int RM, int RN, bool XM, bool TA, bool TB, bool ACC,
          bool PARTIAL>
__global__ void __launch_bounds__((BM / RM) * (BN / RN))
dd_gemm_kernel(GemmParams p) {
  __shared__ DDTileSmem<BM, BN, BK> sm;
  int bi, bj;
  if (!tile_coords(p, bi, bj)) return;     // a tile outside the triangle
  const int64_t i0 = (int64_t)bi * BM;
  const int64_t j0 = (int64_t)bj * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * p.kchunk;
  const int64_t kend = (kbeg + p.kchunk < p.k) ? kbeg + p.kchunk : p.k;
  double ch[RM][RN], cl[RM][RN];
  dd_tile_mainloop<BM, BN, BK, RM, RN, TA, TB, ACC, XM>(p, i0, j0, kbeg, kend, sm, ch, cl);
  dd_tile_epilogue<BM, BN, RM, RN, PARTIAL>(p, i0, j0, (int)blockIdx.z, ch, cl);
}

// Persistent grouped kernel of the request server: a fixed grid walks a list
// of (request, tile) work items (sorted longest first), workgroup g taking
// items g, g + G, g + 2G, ...  Each item runs exactly the steps of
// dd_gemm_kernel for that request's flags, so a request's result is bit-
// identical to a standalone call with the same tile.  The item count is read
// from the device header, so one captured launch serves every group.
template <int BM, int BN, int BK, int RM, int RN, bool XM>
__global__ void __launch_bounds__((BM / RM) * (BN / RN))
dd_grouped_kernel(const char* __restrict__ base, const ServeReq* __restrict__ reqs,
                  const int* __restrict__ counts, const int* __restrict__ items_offset,
                  int which) {
  __shared__ DDTileSmem<BM, BN, BK> sm;
  // the item lists of the tile shapes follow each other after the requests
  const ServeItem* items = (const ServeItem*)(base + *items_offset);
  int first = 0;
  for (int c = 0; c < which; ++c) first += counts[c];
  const int n = counts[which];
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const ServeItem it = items[first + w];
    const GemmParams p = reqs[it.req].p;
    const int flags = reqs[it.req].flags;
    const int64_t i0 = (int64_t)it.bi * BM;
    const int64_t j0 = (int64_t)it.bj * BN;
    double ch[RM][RN], cl[RM][RN];
    switch (flags & 3) {
      case 0: dd_tile_mainloop<BM, BN, BK, RM, RN, false, false, false, XM>(p, i0, j0, 0, p.k, sm, ch, cl); break;
      case 1: dd_tile_mainloop<BM, BN, BK, RM, RN, true, false, false, XM>(p, i0, j0, 0, p.k, sm, ch, cl); break;
      case 2: dd_tile_mainloop<BM, BN, BK, RM, RN, false, true, false, XM>(p, i0, j0, 0, p.k, sm, ch, cl); break;
      default: dd_tile_mainloop<BM, BN, BK, RM, RN, true, true, false, XM>(p, i0, j0, 0, p.k, sm, ch, cl); break;
    }
    dd_tile_epilogue<BM, BN, RM, RN, false>(p, i0, j0, 0, ch, cl);
    __syncthreads();
  }
}

// Add the S k-split partials of every entry in a fixed order and apply the
// alpha / beta update.  One thread per entry: partial s of consecutive
// entries is one coalesced load per wave, and the S partials (S a power of
// two) are summed in a balanced pairwise tree -- ((p0 + p1) + (p2 + p3)) +
// ... -- by a carry-save stack of at most six pending sums: the sum of the
// partials seen so far is held as sums over runs of 2^j partials, and a new
// run is merged with the pending one of its size before it is pushed (the
// earlier run always the left operand).  The order does not depend on the
// schedule, so the result is deterministic.  S is a template parameter, so
// the loop unrolls and the stack stays in registers.
template <int S>
__global__ void __launch_bounds__(256) dd_splitk_reduce(GemmParams p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = p.m * p.n;
  if (e >= total) return;
  const int64_t i = e % p.m, j = e / p.m;
  if (p.tri == 1 && i > j) return;
  if (p.tri == 2 && i < j) return;
  ddv st[7];
  int depth = 0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    ddv v{p.w_hi[(int64_t)s * total + e], p.w_lo[(int64_t)s * total + e]};
    // partial s closes a run of 2^t partials for every trailing one bit t of s + 1
#pragma unroll
    for (int t = s + 1; (t & 1) == 0; t >>= 1) v = dd_add(st[--depth], v);
    st[depth++] = v;
  }
  const ddv v = st[0];
  ddv r = dd_mul(ddv{p.alpha_hi, p.alpha_lo}, v);
  const int64_t ci = i + j * p.ldc;
  if (!p.beta_zero) r = dd_add(r, dd_mul(ddv{p.beta_hi, p.beta_lo}, ddv{p.c_hi[ci], p.c_lo[ci]}));
  p.c_hi[ci] = r.hi;
  p.c_lo[ci] = r.lo;
}

// C <- beta * C on the whole matrix (tri 0) or one triangle; beta = 0 writes
// +0 without reading C.  Used when alpha = 0 or k = 0.
__global__ void __launch_bounds__(256) dd_scale_kernel(GemmParams p) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= p.m * p.n) return;
  const int64_t i = gid % p.m, j = gid / p.m;
  if (p.tri == 1 && i > j) return;
  if (p.tri == 2 && i < j) return;
  const int64_t ci = i + j * p.ldc;
  ddv r{0.0, 0.0};
  if (!p.beta_zero) r = dd_mul(ddv{p.beta_hi, p.beta_lo}, ddv{p.c_hi[ci], p.c_lo[ci]});
  p.c_hi[ci] = r.hi;
  p.c_lo[ci] = r.lo;
}

// {hi, lo} pairs (QD's dd_real layout) <-> separate hi / lo planes.
__global__ void __launch_bounds__(256)
dd_split_pairs(const double* __restrict__ pairs, double* __restrict__ hi, double* __restrict__ lo,
               int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 v = reinterpret_cast<const double2*>(pairs)[i];
  hi[i] = v.x;
  lo[i] = v.y;
}

__global__ void __launch_bounds__(256)
dd_join_pairs(const double* __restrict__ hi, const double* __restrict__ lo,
              double* __restrict__ pairs, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  reinterpret_cast<double2*>(pairs)[i] = make_double2(hi[i], lo[i]);
}

hipError_t launch_split_pairs(const double* pairs, double* hi, double* lo, int64_t n,
                              hipStream_t st) {
  hipLaunchKernelGGL(dd_split_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pairs,
                     hi, lo, n);
  return hipGetLastError();
}

hipError_t launch_join_pairs(const double* hi, const double* lo, double* pairs, int64_t n,
                             hipStream_t st) {
  hipLaunchKernelGGL(dd_join_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, hi, lo,
                     pairs, n);
  return hipGetLastError();
}

// ---- tile table and launchers ------------------------------------------------

// id, BM, BN, BK, RM, RN, XM  (threads = (BM/RM) * (BN/RN); XM: cross terms of
// the lean madd on the FP64 matrix cores)
#define MPDD_TILES(X)         \
  X(0, 64, 64, 16, 4, 4, 0)   \
  X(1, 64, 64, 8, 4, 4, 0)    \
  X(2, 32, 32, 16, 2, 2, 0)   \
  X(3, 128, 64, 8, 8, 4, 0)   \
  X(4, 64, 64, 16, 4, 4, 1)

static const TileInfo kTiles[] = {
#define X(id, bm, bn, bk, rm, rn, xm) {bm, bn, bk, (bm / rm) * (bn / rn)},
    MPDD_TILES(X)
#undef X
};

int tile_count() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
const TileInfo* tile_info(int id) {
  return (id >= 0 && id < tile_count()) ? &kTiles[id] : nullptr;
}

template <int BM, int BN, int BK, int RM, int RN, bool XM, bool TA, bool TB, bool ACC>
static hipError_t launch_t(const GemmParams& p, int nblocks, int splitk, hipStream_t st) {
  dim3 grid(nblocks, 1, splitk), block((BM / RM) * (BN / RN));
  if (splitk > 1)
    hipLaunchKernelGGL((dd_gemm_kernel<BM, BN, BK, RM, RN, XM, TA, TB, ACC, true>), grid, block,
                       0, st, p);
  else
    hipLaunchKernelGGL((dd_gemm_kernel<BM, BN, BK, RM, RN, XM, TA, TB, ACC, false>), grid, block,
                       0, st, p);
  return hipGetLastError();
}

template <int BM, int BN, int BK, int RM, int RN, bool XM>
static hipError_t launch_ops(const GemmParams& p, bool ta, bool tb, bool acc, int nblocks,
                             int splitk, hipStream_t st) {
#define L(TA, TB, AC) return launch_t<BM, BN, BK, RM, RN, XM, TA, TB, AC>(p, nblocks, splitk, st)
  if (acc) {
    if (!ta && !tb) L(false, false, true);
    if (!ta && tb) L(false, true, true);
    if (ta && !tb) L(true, false, true);
    L(true, true, true);
  }
  if (!ta && !tb) L(false, false, false);
  if (!ta && tb) L(false, true, false);
  if (ta && !tb) L(true, false, false);
  L(true, true, false);
#undef L
}

hipError_t launch_gemm(int tile, const GemmParams& p, bool ta, bool tb, bool accurate,
                       int splitk, hipStream_t st) {
  const TileInfo* t = tile_info(tile);
  if (!t) return hipErrorInvalidValue;
  int nblocks;
  if (p.tri == 0) {
    nblocks = p.tiles_m * p.tiles_n;
  } else if ((p.tiles_m & 7) == 0) {           // 8 x 8 blocks over the triangle
    const int s8 = p.tiles_m >> 3;
    nblocks = 64 * (s8 * (s8 + 1) / 2);
  } else {
    nblocks = p.tiles_m * (p.tiles_m + 1) / 2;
  }
  switch (tile) {
#define X(id, bm, bn, bk, rm, rn, xm) \
  case id: return launch_ops<bm, bn, bk, rm, rn, xm != 0>(p, ta, tb, accurate, nblocks, splitk, st);
    MPDD_TILES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_grouped_list(int tile, const char* base, const ServeReq* reqs,
                               const int* counts, const int* items_offset, int which, int grid,
                               hipStream_t st) {
  switch (tile) {
#define X(id, bm, bn, bk, rm, rn, xm)                                                           \
  case id:                                                                                      \
    hipLaunchKernelGGL((dd_grouped_kernel<bm, bn, bk, rm, rn, xm != 0>), dim3(grid),            \
                       dim3((bm / rm) * (bn / rn)), 0, st, base, reqs, counts, items_offset,    \
                       which);                                                                  \
    return hipGetLastError();
    MPDD_TILES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_splitk_reduce(const GemmParams& p, int splitk, hipStream_t st) {
  const int64_t threads = p.m * p.n;
  const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
  switch (splitk) {
    case 2: hipLaunchKernelGGL(dd_splitk_reduce<2>, grid, block, 0, st, p); break;
    case 4: hipLaunchKernelGGL(dd_splitk_reduce<4>, grid, block, 0, st, p); break;
    case 8: hipLaunchKernelGGL(dd_splitk_reduce<8>, grid, block, 0, st, p); break;
    case 16: hipLaunchKernelGGL(dd_splitk_reduce<16>, grid, block, 0, st, p); break;
    case 32: hipLaunchKernelGGL(dd_splitk_reduce<32>, grid, block, 0, st, p); break;
    case 64: hipLaunchKernelGGL(dd_splitk_reduce<64>, grid, block, 0, st, p); break;
    default: return hipErrorInvalidValue;   // the callers split into 2 .. 64 (powers of two)
  }
  return hipGetLastError();
}

hipError_t launch_scale(const GemmParams& p, hipStream_t st) {
  const int64_t total = p.m * p.n;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(dd_scale_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p);
  return hipGetLastError();
}

}  // namespace mpdd

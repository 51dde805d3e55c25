// kernels.hpp -- launch interface between the C-ABI layer (mpdd.cpp) and the
// HIP kernels.  Internal to libmpdd.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mpdd {

// Arguments of one plain dd update, passed by value to the kernels.
struct GemmParams {
  int64_t m, n, k;
  double alpha_hi, alpha_lo, beta_hi, beta_lo;
  const double *a_hi, *a_lo;
  int64_t lda;
  const double *b_hi, *b_lo;
  int64_t ldb;
  double *c_hi, *c_lo;
  int64_t ldc;
  double *w_hi, *w_lo;  // k-split partial sums, [z][j*m + i]
  int64_t kchunk;       // k-range per k-split slice (multiple of the tile depth)
  int tiles_m, tiles_n;
  int tri;              // 0 full matrix, 1 upper triangle, 2 lower triangle
  int beta_zero;        // C is not read
};

// One request of a served group: its update (kchunk = k, no split) and the
// op flags (bit 0: op(A) transposed, bit 1: op(B) transposed).
struct ServeReq {
  GemmParams p;
  int flags;
  int pad_;
};

// One work item of a group: a C tile of a request.
struct ServeItem {
  int req;
  int bi, bj;
};

struct TileInfo {
  int bm, bn, bk, threads;
};

int tile_count();
const TileInfo* tile_info(int id);

hipError_t launch_gemm(int tile, const GemmParams& p, bool ta, bool tb, bool accurate,
                       int splitk, hipStream_t st);
hipError_t launch_splitk_reduce(const GemmParams& p, int splitk, hipStream_t st);
// Persistent grouped kernel over the `which`-th item list: counts[c] items per
// tile shape, lists stored back to back starting at base + *items_offset
// (counts and offset are read on the device, so a captured launch serves
// every group).
hipError_t launch_grouped_list(int tile, const char* base, const ServeReq* reqs,
                               const int* counts, const int* items_offset, int which, int grid,
                               hipStream_t st);
hipError_t launch_scale(const GemmParams& p, hipStream_t st);

// Complex dd epilogue of Cgemm (complex.hip): C <- alpha P + beta C when
// use_p, else C <- beta C; beta_zero: C is not read.  alpha / beta are
// {re.hi, re.lo, im.hi, im.lo}.
struct CEpilogue {
  int64_t m, n;
  double alpha[4], beta[4];
  const double *p_rh, *p_rl, *p_ih, *p_il;
  int64_t ldp;
  double *c_rh, *c_rl, *c_ih, *c_il;
  int64_t ldc;
  int use_p, beta_zero;
  // three_m: p_r = R1, p_i = R2, q = R3; P = (R1 - R2) + i (R3 - R1 - R2)
  const double *q_h, *q_l;
  int three_m;
};
hipError_t launch_cgemm_epilogue(const CEpilogue& p, hipStream_t st);
// out = x + s y elementwise over a rows x cols matrix (x, y: hi / lo planes
// with leading dimension ld; out compact, ld = rows), in dd (s = +-1).
hipError_t launch_dd_axpy_planes(const double* x_hi, const double* x_lo, const double* y_hi,
                                 const double* y_lo, int64_t ld, double s, int64_t rows,
                                 int64_t cols, double* o_hi, double* o_lo, hipStream_t st);

// Quad-double Rgemm (qd.hip): four planes per matrix, alpha / beta as
// {x0, x1, x2, x3}.  scale_only: C <- beta C (alpha = 0 or k = 0);
// beta_zero: C is not read.
struct QgemmParams {
  int64_t m, n, k;
  double alpha[4], beta[4];
  const double* a[4];
  int64_t lda;
  const double* b[4];
  int64_t ldb;
  double* c[4];
  int64_t ldc;
  int beta_zero, scale_only;
};
hipError_t launch_qgemm(const QgemmParams& p, bool ta, bool tb, hipStream_t st);

// Cholesky diagonal block (potrf.hip): factor the jb x jb block (jb <= 64)
// read from s (ld lds) in the lower view (upper = 1: the block holds U, read
// transposed), write the factor's triangle to a (ld lda) and the inverse of
// the lower-view factor to w (ld jb, zero upper part).  *info is the
// factorisation's failure word: if it is already non-zero the kernel does
// nothing; if a pivot of this block fails it becomes offset + the 1-based
// order of that pivot within the block.
hipError_t launch_potf2_block(const double* s_hi, const double* s_lo, int64_t lds, double* a_hi,
                              double* a_lo, int64_t lda, int jb, int upper, double* w_hi,
                              double* w_lo, long long* info, long long offset, hipStream_t st);
// {hi, lo} pairs <-> hi / lo planes (n elements).
hipError_t launch_split_pairs(const double* pairs, double* hi, double* lo, int64_t n,
                              hipStream_t st);
hipError_t launch_join_pairs(const double* hi, const double* lo, double* pairs, int64_t n,
                             hipStream_t st);

}  // namespace mpdd

namespace mpdd {

// Split-form (Ozaki) Rgemm (ozaki.hip), or with tri = 1 / 2 the upper / lower
// triangle of an Rsyrk (m == n, B == A, tb == !ta).  Returns 0 or an
// MPDD_ERR_* code.
int ozaki_gemm(const void* opts, int tri, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
               double alpha_hi, double alpha_lo, const double* a_hi, const double* a_lo,
               int64_t lda, const double* b_hi, const double* b_lo, int64_t ldb,
               double beta_hi, double beta_lo, double* c_hi, double* c_lo, int64_t ldc,
               hipStream_t st, hipMemPool_t pool);

// Split-form qd Rgemm (ozaki.hip; INT8 slices): alpha, beta four parts each,
// a, b, c four planes each; alpha != 0 and k > 0.  Returns 0 or MPDD_ERR_*.
int ozaki_qgemm(const void* opts, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                const double* alpha, const double* const* a, int64_t lda,
                const double* const* b, int64_t ldb, const double* beta, int beta_zero,
                double* const* c, int64_t ldc, hipStream_t st, hipMemPool_t pool);

// Split-form building blocks (ozaki.hip).
int ozaki_split_entry(int algo, bool trans, int64_t rows, int64_t k, const double* hi,
                      const double* lo, int64_t ld, int nslices, int wfirst, int w, int* exps,
                      void* slices, int64_t ldq, int64_t rows_p, hipStream_t st, hipMemPool_t pool);
int ozaki_digit_widths(int algo, int64_t k, int nslices, int* wfirst, int* w);

}  // namespace mpdd

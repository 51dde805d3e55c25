// host_api.cpp -- MPBLAS-shaped host entry points: dd_real arrays in host
// memory, laid out as QD lays them out ({hi, lo} pairs, column-major), as the
// manual's MPBLAS Rgemm / Rsyrk take them (section "How to use reference
// MPBLAS"; the CUDA dd library of section "CUDA accelerated MPBLAS" is linked
// in place of the CPU one behind the same prototype).  The call copies the
// operands to the device, splits them into hi/lo planes, runs the device
// Rgemm / Rsyrk, interleaves C again and copies it back; it returns when C
// is complete, like the CPU routine.  Rgemm pipelines the copies of column
// chunks of B and C with the products of the chunks before them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "../../include/mpdd.h"
#include "kernels.hpp"

namespace {

bool lsame(const char* s, char ref) {
  if (!s) return false;
  char c = s[0];
  if (c >= 'a' && c <= 'z') c = (char)(c - 'a' + 'A');
  return c == ref;
}

bool dd_zero(mpdd_dd x) { return x.hi == 0.0 && x.lo == 0.0; }
bool dd_one(mpdd_dd x) { return x.hi == 1.0 && x.lo == 0.0; }

// Device scratch for one call: interleaved staging + hi/lo planes.
struct Staged {
  void* base = nullptr;
  double *hi = nullptr, *lo = nullptr;
  mpdd_dd* pairs = nullptr;
  size_t n = 0;
};

int stage_alloc(Staged& s, size_t elems, hipStream_t st) {
  s.n = elems;
  if (elems == 0) return 0;
  const size_t bytes = elems * (sizeof(mpdd_dd) + 2 * sizeof(double));
  if (hipMallocAsync(&s.base, bytes, st) != hipSuccess) return MPDD_ERR_ALLOC;
  s.pairs = (mpdd_dd*)s.base;
  s.hi = (double*)((char*)s.base + elems * sizeof(mpdd_dd));
  s.lo = s.hi + elems;
  return 0;
}

int upload(Staged& s, const mpdd_dd* host, hipStream_t st) {
  if (s.n == 0) return 0;
  if (hipMemcpyAsync(s.pairs, host, s.n * sizeof(mpdd_dd), hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return MPDD_ERR_HIP;
  return mpdd::launch_split_pairs((const double*)s.pairs, s.hi, s.lo, (int64_t)s.n, st) ==
                 hipSuccess
             ? 0
             : MPDD_ERR_HIP;
}

int download(Staged& s, mpdd_dd* host, hipStream_t st) {
  if (s.n == 0) return 0;
  if (mpdd::launch_join_pairs(s.hi, s.lo, (double*)s.pairs, (int64_t)s.n, st) != hipSuccess)
    return MPDD_ERR_HIP;
  if (hipMemcpyAsync(host, s.pairs, s.n * sizeof(mpdd_dd), hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return MPDD_ERR_HIP;
  return 0;
}

int finish(Staged* bufs, int nb, int rc, hipStream_t st) {
  for (int i = 0; i < nb; ++i)
    if (bufs[i].base) (void)hipFreeAsync(bufs[i].base, st);
  const hipError_t e = hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  if (rc != 0) return rc;
  return e == hipSuccess ? 0 : MPDD_ERR_HIP;
}

}  // namespace

extern "C" {

int mpdd_Rgemm_host(mpdd_handle h, const char* transa, const char* transb, mpdd_int m, mpdd_int n,
                    mpdd_int k, mpdd_dd alpha, const mpdd_dd* A, mpdd_int lda, const mpdd_dd* B,
                    mpdd_int ldb, mpdd_dd beta, mpdd_dd* C, mpdd_int ldc) {
  // BLAS argument checks before any allocation or copy (same codes as the
  // device routine, which checks again)
  const bool nota = lsame(transa, 'N'), notb = lsame(transb, 'N');
  const mpdd_int nrowa = nota ? m : k, ncola = nota ? k : m;
  const mpdd_int nrowb = notb ? k : n;
  if (!nota && !lsame(transa, 'T') && !lsame(transa, 'C')) return 1;
  if (!notb && !lsame(transb, 'T') && !lsame(transb, 'C')) return 2;
  if (m < 0) return 3;
  if (n < 0) return 4;
  if (k < 0) return 5;
  if (lda < std::max<mpdd_int>(1, nrowa)) return 8;
  if (ldb < std::max<mpdd_int>(1, nrowb)) return 10;
  if (ldc < std::max<mpdd_int>(1, m)) return 13;
  if (!h) return MPDD_ERR_HANDLE;
  if (m == 0 || n == 0 || ((dd_zero(alpha) || k == 0) && dd_one(beta))) return 0;
  const bool use_ab = !dd_zero(alpha) && k > 0;
  if (!C || (use_ab && (!A || !B))) return MPDD_ERR_ARG;

  // Pipelined over column chunks of C: while chunk c is multiplied on the
  // compute stream, chunk c+1's operands are copied in and chunk c-1's result
  // copied out on the copy stream.  A is copied in once, first.
  const int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(8, n / 512));
  const int64_t cw = (n + nchunk - 1) / nchunk;          // columns per chunk
  hipStream_t sc = nullptr, sx = nullptr;
  hipEvent_t ev_in[2] = {nullptr, nullptr}, ev_out[2] = {nullptr, nullptr};
  bool ok = hipStreamCreateWithFlags(&sc, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&sx, hipStreamNonBlocking) == hipSuccess;
  for (int t = 0; t < 2 && ok; ++t)
    ok = hipEventCreateWithFlags(&ev_in[t], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&ev_out[t], hipEventDisableTiming) == hipSuccess;
  Staged sa, sbuf[2], scb[2];
  int rc = ok ? 0 : MPDD_ERR_HIP;
  // B chunk: columns j0.. of op(B): for 'N' the columns of B, for 'T' its rows
  const size_t nb_chunk = use_ab ? (notb ? (size_t)ldb * cw : (size_t)cw * k) : 0;
  const size_t nc_chunk = (size_t)ldc * cw;
  if (!rc && use_ab) rc = stage_alloc(sa, (size_t)lda * (size_t)ncola, sx);
  for (int t = 0; t < 2 && !rc; ++t) {
    rc = stage_alloc(sbuf[t], nb_chunk, sx);
    if (!rc) rc = stage_alloc(scb[t], nc_chunk, sx);
  }
  if (!rc && use_ab) rc = upload(sa, A, sx);
  auto upload_chunk = [&](int64_t c) -> int {
    const int64_t j0 = c * cw, w = std::min<int64_t>(cw, n - j0);
    const int t = (int)(c & 1);
    if (use_ab) {
      if (notb) {
        sbuf[t].n = (size_t)ldb * w;
        if (int r = upload(sbuf[t], B + (size_t)j0 * ldb, sx)) return r;
      } else {
        // rows j0 .. j0+w of B (k columns): a 2-D copy into a compact w x k block
        sbuf[t].n = (size_t)w * k;
        if (hipMemcpy2DAsync(sbuf[t].pairs, w * sizeof(mpdd_dd), B + j0, ldb * sizeof(mpdd_dd),
                             w * sizeof(mpdd_dd), k, hipMemcpyHostToDevice, sx) != hipSuccess ||
            mpdd::launch_split_pairs((const double*)sbuf[t].pairs, sbuf[t].hi, sbuf[t].lo,
                                     (int64_t)sbuf[t].n, sx) != hipSuccess)
          return MPDD_ERR_HIP;
      }
    }
    scb[t].n = (size_t)ldc * w;
    if (int r = upload(scb[t], C + (size_t)j0 * ldc, sx)) return r;
    return hipEventRecord(ev_in[t], sx) == hipSuccess ? 0 : MPDD_ERR_HIP;
  };
  auto multiply_chunk = [&](int64_t c) -> int {
    const int64_t j0 = c * cw, w = std::min<int64_t>(cw, n - j0);
    const int t = (int)(c & 1);
    if (hipStreamWaitEvent(sc, ev_in[t], 0) != hipSuccess) return MPDD_ERR_HIP;
    const mpdd_int ldbc = notb ? ldb : (mpdd_int)w;
    int r = mpdd_Rgemm(h, transa, transb, m, w, k, alpha, sa.hi, sa.lo, lda, sbuf[t].hi,
                       sbuf[t].lo, ldbc, beta, scb[t].hi, scb[t].lo, ldc, (void*)sc);
    if (r) return r;
    if (mpdd::launch_join_pairs(scb[t].hi, scb[t].lo, (double*)scb[t].pairs, (int64_t)scb[t].n,
                                sc) != hipSuccess ||
        hipEventRecord(ev_out[t], sc) != hipSuccess)
      return MPDD_ERR_HIP;
    return 0;
  };
  auto download_chunk = [&](int64_t c) -> int {
    const int64_t j0 = c * cw;
    const int t = (int)(c & 1);
    if (hipStreamWaitEvent(sx, ev_out[t], 0) != hipSuccess ||
        hipMemcpyAsync(C + (size_t)j0 * ldc, scb[t].pairs, scb[t].n * sizeof(mpdd_dd),
                       hipMemcpyDeviceToHost, sx) != hipSuccess ||
        hipStreamSynchronize(sx) != hipSuccess)
      return MPDD_ERR_HIP;
    return 0;
  };
  if (!rc) rc = upload_chunk(0);
  if (!rc) rc = multiply_chunk(0);
  for (int64_t c = 1; c < nchunk && !rc; ++c) {
    // buffer c & 1 was last used by chunk c-2, downloaded (synchronously)
    // in the previous iteration
    rc = upload_chunk(c);
    if (!rc) rc = multiply_chunk(c);
    if (!rc) rc = download_chunk(c - 1);
  }
  if (!rc) rc = download_chunk(nchunk - 1);
  // release (after both streams have drained; the scratch was allocated
  // stream-ordered on the copy stream)
  if (sc) (void)hipStreamSynchronize(sc);
  Staged* all[5] = {&sa, &sbuf[0], &sbuf[1], &scb[0], &scb[1]};
  for (Staged* b : all)
    if (b->base) (void)hipFreeAsync(b->base, sx);
  if (sx && hipStreamSynchronize(sx) != hipSuccess && !rc) rc = MPDD_ERR_HIP;
  for (int t = 0; t < 2; ++t) {
    if (ev_in[t]) (void)hipEventDestroy(ev_in[t]);
    if (ev_out[t]) (void)hipEventDestroy(ev_out[t]);
  }
  if (sc) (void)hipStreamDestroy(sc);
  if (sx) (void)hipStreamDestroy(sx);
  return rc;
}

int mpdd_Rsyrk_host(mpdd_handle h, const char* uplo, const char* trans, mpdd_int n, mpdd_int k,
                    mpdd_dd alpha, const mpdd_dd* A, mpdd_int lda, mpdd_dd beta, mpdd_dd* C,
                    mpdd_int ldc) {
  const bool upper = lsame(uplo, 'U');
  const bool nt = lsame(trans, 'N');
  const mpdd_int nrowa = nt ? n : k, ncola = nt ? k : n;
  if (!upper && !lsame(uplo, 'L')) return 1;
  if (!nt && !lsame(trans, 'T') && !lsame(trans, 'C')) return 2;
  if (n < 0) return 3;
  if (k < 0) return 4;
  if (lda < std::max<mpdd_int>(1, nrowa)) return 7;
  if (ldc < std::max<mpdd_int>(1, n)) return 10;
  if (!h) return MPDD_ERR_HANDLE;
  if (n == 0 || ((dd_zero(alpha) || k == 0) && dd_one(beta))) return 0;
  const bool use_a = !dd_zero(alpha) && k > 0;
  if (!C || (use_a && !A)) return MPDD_ERR_ARG;
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return MPDD_ERR_HIP;
  Staged bufs[2];
  int rc = 0;
  const size_t na = use_a ? (size_t)lda * (size_t)ncola : 0;
  const size_t nc = (size_t)ldc * (size_t)n;
  if (!rc) rc = stage_alloc(bufs[0], na, st);
  if (!rc) rc = stage_alloc(bufs[1], nc, st);
  if (!rc) rc = upload(bufs[0], A, st);
  if (!rc) rc = upload(bufs[1], C, st);
  if (!rc)
    rc = mpdd_Rsyrk(h, uplo, trans, n, k, alpha, bufs[0].hi, bufs[0].lo, lda, beta, bufs[1].hi,
                    bufs[1].lo, ldc, (void*)st);
  if (!rc) rc = download(bufs[1], C, st);
  return finish(bufs, 2, rc, st);
}

}  // extern "C"

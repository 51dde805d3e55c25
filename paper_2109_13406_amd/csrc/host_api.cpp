// host_api.cpp -- MPBLAS-shaped host entry points: dd_real arrays in host
// memory, laid out as QD lays them out ({hi, lo} pairs, column-major), as the
// manual's MPBLAS Rgemm / Rsyrk take them (section "How to use reference
// MPBLAS"; the CUDA dd library of section "CUDA accelerated MPBLAS" is linked
// in place of the CPU one behind the same prototype).  The call copies the
// operands to the device, splits them into hi/lo planes, runs the device
// Rgemm / Rsyrk, interleaves C again and copies it back; it returns when C
// is complete, like the CPU routine.  Rgemm pipelines the copies of column
// chunks of B and C with the products of the chunks before them and with the
// copies back of the chunks before those.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/mpdd.h"
#include "extent.hpp"
#include "kernels.hpp"
#include "tuner.hpp"

namespace mpdd {

// Copies between pageable host memory and the device through a ring of
// pinned buffers.  A DMA from or to pageable memory runs at about half the
// pinned rate (measured on MI355X: 29 / 17 GB/s H2D / D2H against 58 / 57),
// so each piece is copied by host threads into a pinned buffer, and the DMA
// of one piece overlaps the host copy of the next.  Two stagers per handle
// (one per copy direction, so that copies in and copies back can run at
// once), created by its first host-pointer call; the calls on a handle are
// serialised.
class HostStager {
 public:
  static constexpr int kSlots = 4;
  static constexpr size_t kPiece = size_t(16) << 20;   // bytes per pinned buffer
  static constexpr int kThreads = 4;                   // host copy threads (with the caller)

  int init() {
    for (int i = 0; i < kSlots; ++i) {
      if (hipHostMalloc(&slot_[i], kPiece, hipHostMallocDefault) != hipSuccess) return MPDD_ERR_ALLOC;
      if (hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming) != hipSuccess) return MPDD_ERR_HIP;
    }
    try {
      for (int i = 1; i < kThreads; ++i) workers_.emplace_back([this, i] { work(i); });
    } catch (...) {               // no thread: the destructor stops the ones started
      return MPDD_ERR_ALLOC;
    }
    return 0;
  }

  ~HostStager() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (std::thread& t : workers_) t.join();
    for (int i = 0; i < kSlots; ++i) {
      if (pending_[i]) (void)hipEventSynchronize(ev_[i]);
      if (ev_[i]) (void)hipEventDestroy(ev_[i]);
      if (slot_[i]) (void)hipHostFree(slot_[i]);
    }
  }

  // host -> device; returns once every piece is enqueued on st (the pinned
  // buffers are then reused only after their copy has completed)
  int h2d(void* dev, const void* host, size_t bytes, hipStream_t st) {
    for (size_t off = 0; off < bytes; off += kPiece) {
      const size_t n = std::min(kPiece, bytes - off);
      const int s = take_slot();
      if (s < 0) return MPDD_ERR_HIP;
      copy(slot_[s], (const char*)host + off, n);
      if (hipMemcpyAsync((char*)dev + off, slot_[s], n, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipEventRecord(ev_[s], st) != hipSuccess)
        return MPDD_ERR_HIP;
      pending_[s] = true;
    }
    return 0;
  }

  // device -> host, in stream order on st; returns when the host holds the data
  int d2h(void* host, const void* dev, size_t bytes, hipStream_t st) {
    const size_t npiece = (bytes + kPiece - 1) / kPiece;
    std::vector<int> slot_of(npiece, -1);
    auto enqueue = [&](size_t p) -> int {
      const size_t off = p * kPiece, n = std::min(kPiece, bytes - off);
      const int s = take_slot();
      if (s < 0) return MPDD_ERR_HIP;
      if (hipMemcpyAsync(slot_[s], (const char*)dev + off, n, hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipEventRecord(ev_[s], st) != hipSuccess)
        return MPDD_ERR_HIP;
      pending_[s] = true;
      slot_of[p] = s;
      return 0;
    };
    for (size_t p = 0; p < npiece && p < (size_t)kSlots - 1; ++p)
      if (int r = enqueue(p)) return r;
    for (size_t p = 0; p < npiece; ++p) {
      if (p + kSlots - 1 < npiece)
        if (int r = enqueue(p + kSlots - 1)) return r;
      const int s = slot_of[p];
      if (hipEventSynchronize(ev_[s]) != hipSuccess) return MPDD_ERR_HIP;
      pending_[s] = false;
      const size_t off = p * kPiece;
      copy((char*)host + off, slot_[s], std::min(kPiece, bytes - off));
    }
    return 0;
  }

 private:
  // the next ring buffer, once its previous copy has completed
  int take_slot() {
    const int s = next_;
    next_ = (next_ + 1) % kSlots;
    if (pending_[s]) {
      if (hipEventSynchronize(ev_[s]) != hipSuccess) return -1;
      pending_[s] = false;
    }
    return s;
  }

  // memcpy split over the caller and the workers
  void copy(void* dst, const void* src, size_t n) {
    const size_t part = ((n + kThreads - 1) / kThreads + 63) / 64 * 64;
    {
      std::lock_guard<std::mutex> lk(mu_);
      dst_ = (char*)dst;
      src_ = (const char*)src;
      n_ = n;
      part_ = part;
      remaining_ = kThreads - 1;
      ++gen_;
    }
    cv_.notify_all();
    copy_part(0);
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return remaining_ == 0; });
  }

  void copy_part(int i) {
    const size_t b = std::min(n_, (size_t)i * part_), e = std::min(n_, b + part_);
    if (e > b) std::memcpy(dst_ + b, src_ + b, e - b);
  }

  void work(int i) {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return gen_ != seen; });
      seen = gen_;
      if (stop_) return;
      lk.unlock();
      copy_part(i);
      lk.lock();
      if (--remaining_ == 0) cv_done_.notify_one();
    }
  }

  void* slot_[kSlots] = {};
  hipEvent_t ev_[kSlots] = {};
  bool pending_[kSlots] = {};
  int next_ = 0;
  std::vector<std::thread> workers_;
  std::mutex mu_;
  std::condition_variable cv_, cv_done_;
  uint64_t gen_ = 0;
  bool stop_ = false;
  char* dst_ = nullptr;
  const char* src_ = nullptr;
  size_t n_ = 0, part_ = 0;
  int remaining_ = 0;
};

}  // namespace mpdd

void destroy_stager(mpdd::HostStager* st) { delete st; }

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

int stage_alloc(Staged& s, size_t elems, hipStream_t st, hipMemPool_t pool) {
  s.n = elems;
  if (elems == 0) return 0;
  const size_t bytes = elems * (sizeof(mpdd_dd) + 2 * sizeof(double));
  if (hipMallocFromPoolAsync(&s.base, bytes, pool, st) != hipSuccess) return MPDD_ERR_ALLOC;
  s.pairs = (mpdd_dd*)s.base;
  s.hi = (double*)((char*)s.base + elems * sizeof(mpdd_dd));
  s.lo = s.hi + elems;
  return 0;
}

int upload(Staged& s, const mpdd_dd* host, hipStream_t st, mpdd::HostStager* stg) {
  if (s.n == 0) return 0;
  if (int r = stg->h2d(s.pairs, host, s.n * sizeof(mpdd_dd), st)) return r;
  return mpdd::launch_split_pairs((const double*)s.pairs, s.hi, s.lo, (int64_t)s.n, st) ==
                 hipSuccess
             ? 0
             : MPDD_ERR_HIP;
}

// joins C's planes into pairs and copies them back; returns when the host
// holds them
int download(Staged& s, mpdd_dd* host, hipStream_t st, mpdd::HostStager* stg) {
  if (s.n == 0) return 0;
  if (mpdd::launch_join_pairs(s.hi, s.lo, (double*)s.pairs, (int64_t)s.n, st) != hipSuccess)
    return MPDD_ERR_HIP;
  return stg->d2h(host, s.pairs, s.n * sizeof(mpdd_dd), st);
}

// One of the handle's two stagers (0: copies to the device, 1: copies
// back), created on first use (the caller holds the handle's host-call lock).
int stager_of(mpdd_handle h, mpdd::HostStager*& out, int which = 0) {
  mpdd::HostStager** slot = handle_stager(h, which);
  if (!*slot) {
    auto* st = new (std::nothrow) mpdd::HostStager();
    if (!st) return MPDD_ERR_ALLOC;
    if (int r = st->init()) {
      delete st;
      return r;
    }
    *slot = st;
  }
  out = *slot;
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

int mpdd_Rgemm_host_ex(mpdd_handle h, const mpdd_opts* opts, const char* transa,
                       const char* transb, mpdd_int m, mpdd_int n, mpdd_int k, mpdd_dd alpha,
                       const mpdd_dd* A, mpdd_int lda, const mpdd_dd* B, mpdd_int ldb,
                       mpdd_dd beta, mpdd_dd* C, mpdd_int ldc) {
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
  if (!handle_valid(h)) return MPDD_ERR_HANDLE;
  if (m == 0 || n == 0 || ((dd_zero(alpha) || k == 0) && dd_one(beta))) return 0;
  const bool use_ab = !dd_zero(alpha) && k > 0;
  if (!C || (use_ab && (!A || !B))) return MPDD_ERR_ARG;
  std::lock_guard<std::mutex> host_lock(*handle_host_mutex(h));
  mpdd::HostStager* stg = nullptr;      // copies to the device
  mpdd::HostStager* stg_d = nullptr;    // copies back
  if (int r = stager_of(h, stg, 0)) return r;
  if (int r = stager_of(h, stg_d, 1)) return r;

  // Pipelined over column chunks of C, three chunk buffers in turn: while
  // chunk c is copied in (copy stream, this thread) and multiplied (compute
  // stream), chunk c-1's result is copied out by a helper thread through the
  // second stager on a third stream, so the two copy directions overlap.  A
  // is copied in once; when op(A) = A and the form is a plain one, its
  // columns are k-slices of the product, so chunk 0 is multiplied slice by
  // slice as they arrive (accumulating into C with beta = 1 after the
  // first), and A's copy overlaps that product.
  constexpr int NBUF = 3;
  const int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(8, n / 512));
  const int64_t cw = (n + nchunk - 1) / nchunk;          // columns per chunk
  // (plain forms only: a split form scales each row of op(A) over all of k
  // and sizes its slices or moduli for k, so its chunks take the whole k)
  const bool plain = !opts || opts->algo == MPDD_PLAIN || opts->algo == MPDD_PLAIN_ACCURATE;
  const bool slice_a = use_ab && nota && k >= 1024 && plain;
  const int64_t nks = slice_a ? std::min<int64_t>(8, k / 512) : 1;
  const int64_t kcs = (k + nks - 1) / nks;               // k per slice
  hipStream_t sc = nullptr, sx = nullptr, sd = nullptr;
  hipEvent_t ev_in[NBUF] = {}, ev_out[NBUF] = {};
  hipEvent_t ev_a[8] = {};
  bool ok = hipStreamCreateWithFlags(&sc, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&sx, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&sd, hipStreamNonBlocking) == hipSuccess;
  for (int t = 0; t < NBUF && ok; ++t)
    ok = hipEventCreateWithFlags(&ev_in[t], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&ev_out[t], hipEventDisableTiming) == hipSuccess;
  for (int64_t t = 0; t < nks && slice_a && ok; ++t)
    ok = hipEventCreateWithFlags(&ev_a[t], hipEventDisableTiming) == hipSuccess;
  Staged sa, sbuf[NBUF], scb[NBUF];
  int rc = ok ? 0 : MPDD_ERR_HIP;
  // B chunk: columns j0.. of op(B): for 'N' the columns of B, for 'T' its rows
  const size_t nb_chunk = use_ab ? (notb ? (size_t)ldb * cw : (size_t)cw * k) : 0;
  const size_t nc_chunk = (size_t)ldc * cw;
  if (!rc && use_ab) rc = stage_alloc(sa, mpdd::blas_extent(lda, nrowa, ncola), sx, handle_pool(h));
  for (int t = 0; t < NBUF && !rc; ++t) {
    rc = stage_alloc(sbuf[t], nb_chunk, sx, handle_pool(h));
    if (!rc) rc = stage_alloc(scb[t], nc_chunk, sx, handle_pool(h));
  }
  // the buffers were allocated in stream order on sx: the download stream
  // starts after that
  if (!rc && (hipEventRecord(ev_in[0], sx) != hipSuccess ||
              hipStreamWaitEvent(sd, ev_in[0], 0) != hipSuccess))
    rc = MPDD_ERR_HIP;
  if (!rc && use_ab && !slice_a) rc = upload(sa, A, sx, stg);
  auto upload_chunk = [&](int64_t c) -> int {
    const int64_t j0 = c * cw, w = std::min<int64_t>(cw, n - j0);
    const int t = (int)(c % NBUF);
    if (use_ab) {
      if (notb) {
        sbuf[t].n = mpdd::blas_extent(ldb, k, w);
        if (int r = upload(sbuf[t], B + (size_t)j0 * ldb, sx, stg)) return r;
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
    scb[t].n = mpdd::blas_extent(ldc, m, w);
    if (int r = upload(scb[t], C + (size_t)j0 * ldc, sx, stg)) return r;
    return hipEventRecord(ev_in[t], sx) == hipSuccess ? 0 : MPDD_ERR_HIP;
  };
  auto multiply_chunk = [&](int64_t c) -> int {
    const int64_t j0 = c * cw, w = std::min<int64_t>(cw, n - j0);
    const int t = (int)(c % NBUF);
    if (hipStreamWaitEvent(sc, ev_in[t], 0) != hipSuccess) return MPDD_ERR_HIP;
    const mpdd_int ldbc = notb ? ldb : (mpdd_int)w;
    int r = mpdd_Rgemm_ex(h, opts, transa, transb, m, w, k, alpha, sa.hi, sa.lo, lda,
                          sbuf[t].hi, sbuf[t].lo, ldbc, beta, scb[t].hi, scb[t].lo, ldc,
                          (void*)sc);
    if (r) return r;
    if (mpdd::launch_join_pairs(scb[t].hi, scb[t].lo, (double*)scb[t].pairs, (int64_t)scb[t].n,
                                sc) != hipSuccess ||
        hipEventRecord(ev_out[t], sc) != hipSuccess)
      return MPDD_ERR_HIP;
    return 0;
  };
  // chunk 0 with op(A) = A: slice s of k is columns k0 .. k0+kk of A (one
  // contiguous range) and rows k0 .. k0+kk of op(B)'s chunk
  auto multiply_chunk0_sliced = [&]() -> int {
    const int64_t w = std::min<int64_t>(cw, n);
    if (hipStreamWaitEvent(sc, ev_in[0], 0) != hipSuccess) return MPDD_ERR_HIP;
    const mpdd_int ldbc = notb ? ldb : (mpdd_int)w;
    const mpdd_dd one{1.0, 0.0};
    for (int64_t sl = 0; sl < nks; ++sl) {
      const int64_t k0 = sl * kcs, kk = std::min<int64_t>(kcs, k - k0);
      const size_t off = (size_t)k0 * lda, cnt = mpdd::blas_extent(lda, m, kk);
      if (int r = stg->h2d(sa.pairs + off, A + off, cnt * sizeof(mpdd_dd), sx)) return r;
      if (mpdd::launch_split_pairs((const double*)(sa.pairs + off), sa.hi + off, sa.lo + off,
                                   (int64_t)cnt, sx) != hipSuccess ||
          hipEventRecord(ev_a[sl], sx) != hipSuccess ||
          hipStreamWaitEvent(sc, ev_a[sl], 0) != hipSuccess)
        return MPDD_ERR_HIP;
      const size_t boff = notb ? (size_t)k0 : (size_t)k0 * (size_t)w;
      int r = mpdd_Rgemm_ex(h, opts, transa, transb, m, w, kk, alpha, sa.hi + off,
                            sa.lo + off, lda, sbuf[0].hi + boff, sbuf[0].lo + boff, ldbc,
                            sl == 0 ? beta : one, scb[0].hi, scb[0].lo, ldc, (void*)sc);
      if (r) return r;
    }
    if (mpdd::launch_join_pairs(scb[0].hi, scb[0].lo, (double*)scb[0].pairs, (int64_t)scb[0].n,
                                sc) != hipSuccess ||
        hipEventRecord(ev_out[0], sc) != hipSuccess)
      return MPDD_ERR_HIP;
    return 0;
  };
  // copy chunk c's result back (download stream, second stager)
  auto download_chunk = [&](int64_t c) -> int {
    const int64_t j0 = c * cw;
    const int t = (int)(c % NBUF);
    if (hipStreamWaitEvent(sd, ev_out[t], 0) != hipSuccess) return MPDD_ERR_HIP;
    return stg_d->d2h(C + (size_t)j0 * ldc, scb[t].pairs, scb[t].n * sizeof(mpdd_dd), sd);
  };
  // at most one download in flight on the helper thread; joined before the
  // next one starts (so its buffer, NBUF - 1 chunks back, is free by the time
  // it is filled again) and before anything is released
  std::thread helper;
  int rc_dl = 0;
  int dev = 0;                   // HIP's current device is per thread
  if (!rc && hipGetDevice(&dev) != hipSuccess) rc = MPDD_ERR_HIP;
  auto join_download = [&]() {
    if (helper.joinable()) helper.join();
    if (!rc && rc_dl) rc = rc_dl;
  };
  auto start_download = [&](int64_t c) {
    join_download();
    if (rc) return;
    try {
      helper = std::thread([&, c] {
        rc_dl = hipSetDevice(dev) == hipSuccess ? download_chunk(c) : MPDD_ERR_HIP;
      });
    } catch (...) {              // no thread: copy it back here
      rc = download_chunk(c);
    }
  };
  if (!rc) rc = upload_chunk(0);
  if (!rc) rc = slice_a ? multiply_chunk0_sliced() : multiply_chunk(0);
  for (int64_t c = 1; c < nchunk && !rc; ++c) {
    // buffer c % NBUF was last used by chunk c - NBUF, whose download was
    // joined when chunk c - 1's started
    rc = upload_chunk(c);
    if (!rc) rc = multiply_chunk(c);
    if (!rc) start_download(c - 1);
  }
  join_download();
  if (!rc) rc = download_chunk(nchunk - 1);
  // release (after every stream has drained; the scratch was allocated
  // stream-ordered on the copy stream)
  if (sc) (void)hipStreamSynchronize(sc);
  if (sd) (void)hipStreamSynchronize(sd);
  Staged* all[1 + 2 * NBUF] = {&sa};
  for (int t = 0; t < NBUF; ++t) {
    all[1 + 2 * t] = &sbuf[t];
    all[2 + 2 * t] = &scb[t];
  }
  for (Staged* b : all)
    if (b->base) (void)hipFreeAsync(b->base, sx);
  if (sx && hipStreamSynchronize(sx) != hipSuccess && !rc) rc = MPDD_ERR_HIP;
  for (int t = 0; t < NBUF; ++t) {
    if (ev_in[t]) (void)hipEventDestroy(ev_in[t]);
    if (ev_out[t]) (void)hipEventDestroy(ev_out[t]);
  }
  for (hipEvent_t e : ev_a)
    if (e) (void)hipEventDestroy(e);
  if (sc) (void)hipStreamDestroy(sc);
  if (sx) (void)hipStreamDestroy(sx);
  if (sd) (void)hipStreamDestroy(sd);
  return rc;
}

int mpdd_Rgemm_host(mpdd_handle h, const char* transa, const char* transb, mpdd_int m, mpdd_int n,
                    mpdd_int k, mpdd_dd alpha, const mpdd_dd* A, mpdd_int lda, const mpdd_dd* B,
                    mpdd_int ldb, mpdd_dd beta, mpdd_dd* C, mpdd_int ldc) {
  return mpdd_Rgemm_host_ex(h, nullptr, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C,
                            ldc);
}

int mpdd_Rsyrk_host_ex(mpdd_handle h, const mpdd_opts* opts, const char* uplo,
                       const char* trans, mpdd_int n, mpdd_int k, mpdd_dd alpha,
                       const mpdd_dd* A, mpdd_int lda, mpdd_dd beta, mpdd_dd* C, mpdd_int ldc) {
  const bool upper = lsame(uplo, 'U');
  const bool nt = lsame(trans, 'N');
  const mpdd_int nrowa = nt ? n : k, ncola = nt ? k : n;
  if (!upper && !lsame(uplo, 'L')) return 1;
  if (!nt && !lsame(trans, 'T') && !lsame(trans, 'C')) return 2;
  if (n < 0) return 3;
  if (k < 0) return 4;
  if (lda < std::max<mpdd_int>(1, nrowa)) return 7;
  if (ldc < std::max<mpdd_int>(1, n)) return 10;
  if (!handle_valid(h)) return MPDD_ERR_HANDLE;
  if (n == 0 || ((dd_zero(alpha) || k == 0) && dd_one(beta))) return 0;
  const bool use_a = !dd_zero(alpha) && k > 0;
  if (!C || (use_a && !A)) return MPDD_ERR_ARG;
  std::lock_guard<std::mutex> host_lock(*handle_host_mutex(h));
  mpdd::HostStager* stg = nullptr;
  if (int r = stager_of(h, stg)) return r;
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return MPDD_ERR_HIP;
  Staged bufs[2];
  int rc = 0;
  const size_t na = use_a ? mpdd::blas_extent(lda, nrowa, ncola) : 0;
  const size_t nc = mpdd::blas_extent(ldc, n, n);
  if (!rc) rc = stage_alloc(bufs[0], na, st, handle_pool(h));
  if (!rc) rc = stage_alloc(bufs[1], nc, st, handle_pool(h));
  if (!rc) rc = upload(bufs[0], A, st, stg);
  if (!rc) rc = upload(bufs[1], C, st, stg);
  if (!rc)
    rc = mpdd_Rsyrk_ex(h, opts, uplo, trans, n, k, alpha, bufs[0].hi, bufs[0].lo, lda, beta,
                       bufs[1].hi, bufs[1].lo, ldc, (void*)st);
  if (!rc) rc = download(bufs[1], C, st, stg);
  return finish(bufs, 2, rc, st);
}

int mpdd_Rsyrk_host(mpdd_handle h, const char* uplo, const char* trans, mpdd_int n, mpdd_int k,
                    mpdd_dd alpha, const mpdd_dd* A, mpdd_int lda, mpdd_dd beta, mpdd_dd* C,
                    mpdd_int ldc) {
  return mpdd_Rsyrk_host_ex(h, nullptr, uplo, trans, n, k, alpha, A, lda, beta, C, ldc);
}

}  // extern "C"

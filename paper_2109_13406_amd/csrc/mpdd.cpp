// mpdd.cpp -- the C ABI of libmpdd (declared in include/mpdd.h): argument
// checking, BLAS quick returns, tile / k-split choice and kernel dispatch for
// the plain dd Rgemm and Rsyrk.
//
// Argument checks and quick returns follow the BLAS reference DGEMM / DSYRK
// (the MPLAPACK manual's section "How to use reference MPBLAS" gives Rgemm
// DGEMM's argument list; its MPBLAS quality-assurance section requires error
// codes equal to xerbla's).  Checks run on the host before any HIP call, so
// an invalid call has no side effects at all.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/mpdd.h"
#include "crt.hpp"
#include "kernels.hpp"
#include "tuner.hpp"

using namespace mpdd;

// Static device scratch of the no-allocation entry point (mpdd_Rgemm_noalloc):
// its k-split partial sums live here instead of in a handle's pool, so that
// the call allocates nothing.  Each device that loads the library holds its
// own copy until the process ends.  In host code the name `scratch` is a
// host-side stand-in, not a device address: host code only ever uses the
// address that hipGetSymbolAddress returns for the device (looked up once per
// device by mpdd_create, with the device current, and kept in
// g_static_scratch).
static __device__ __align__(256) char scratch[MPDD_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_scratch_mu;
std::atomic<void*> g_static_scratch[kMaxDevices];   // device -> address of `scratch` on it

// Look up the address of `scratch` on `device`, which must be the current
// device.  Once per device; later calls return at once.
int static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return MPDD_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_static_scratch_mu);
  if (g_static_scratch[device].load(std::memory_order_acquire)) return 0;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
    return MPDD_ERR_HIP;
  g_static_scratch[device].store(p, std::memory_order_release);
  return 0;
}

void* static_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  return g_static_scratch[device].load(std::memory_order_acquire);
}

}  // namespace

struct mpdd_handle_s {
  int device = 0;
  int magic = 0x6d706464;
  TuneTable tune;
  // Stream-ordered scratch (k-split partials, split-form slices, Cgemm
  // planes, Rpotrf panels, host staging) comes from the handle's own pool,
  // which keeps freed memory for the next call instead of returning it to the
  // driver at every synchronisation (1024^3 Rgemm with its k-split partials:
  // 510 -> 449 us per call).  The pool holds its peak size until
  // mpdd_destroy.
  hipMemPool_t pool = nullptr;
  std::mutex host_mu;           // serialises the host-pointer calls on this handle
  // their pinned staging (created on first use): [0] for copies to the
  // device, [1] for copies back, so that the two directions can overlap
  HostStager* stager[2] = {nullptr, nullptr};
};

std::mutex* handle_host_mutex(mpdd_handle_s* h) { return &h->host_mu; }
hipMemPool_t handle_pool(const mpdd_handle_s* h) { return h->pool; }
HostStager** handle_stager(mpdd_handle_s* h, int which) { return &h->stager[which]; }

bool handle_valid(const mpdd_handle_s* h) { return h != nullptr && h->magic == 0x6d706464; }

int handle_device(const mpdd_handle_s* h) { return h ? h->device : 0; }

bool handle_tune_lookup(const mpdd_handle_s* h, int op, bool ta, bool tb, int64_t m, int64_t n,
                        int64_t k, TuneEntry& out) {
  return handle_valid(h) && h->tune.lookup(op, ta, tb, m, n, k, out);
}

namespace {

bool lsame(const char* s, char ref) {
  if (!s) return false;
  char c = s[0];
  if (c >= 'a' && c <= 'z') c = (char)(c - 'a' + 'A');
  return c == ref;
}

bool is_zero(mpdd_dd x) { return x.hi == 0.0 && x.lo == 0.0; }
// The split forms (slices or residues on the matrix cores).
bool split_algo(int a) {
  return a == MPDD_OZAKI_I8 || a == MPDD_OZAKI_F64 || a == MPDD_OZAKI_CRT;
}
bool is_one(mpdd_dd x) { return x.hi == 1.0 && x.lo == 0.0; }

int check_gemm(const char* ta, const char* tb, mpdd_int m, mpdd_int n, mpdd_int k, mpdd_int lda,
               mpdd_int ldb, mpdd_int ldc) {
  const bool nota = lsame(ta, 'N'), notb = lsame(tb, 'N');
  const mpdd_int nrowa = nota ? m : k;
  const mpdd_int nrowb = notb ? k : n;
  if (!nota && !lsame(ta, 'T') && !lsame(ta, 'C')) return 1;
  if (!notb && !lsame(tb, 'T') && !lsame(tb, 'C')) return 2;
  if (m < 0) return 3;
  if (n < 0) return 4;
  if (k < 0) return 5;
  if (lda < std::max<mpdd_int>(1, nrowa)) return 8;
  if (ldb < std::max<mpdd_int>(1, nrowb)) return 10;
  if (ldc < std::max<mpdd_int>(1, m)) return 13;
  return 0;
}

int check_syrk(const char* uplo, const char* trans, mpdd_int n, mpdd_int k, mpdd_int lda,
               mpdd_int ldc) {
  const bool upper = lsame(uplo, 'U');
  const mpdd_int nrowa = lsame(trans, 'N') ? n : k;
  if (!upper && !lsame(uplo, 'L')) return 1;
  if (!lsame(trans, 'N') && !lsame(trans, 'T') && !lsame(trans, 'C')) return 2;
  if (n < 0) return 3;
  if (k < 0) return 4;
  if (lda < std::max<mpdd_int>(1, nrowa)) return 7;
  if (ldc < std::max<mpdd_int>(1, n)) return 10;
  return 0;
}

int hip_status(hipError_t e) { return e == hipSuccess ? 0 : MPDD_ERR_HIP; }

bool handle_ok(mpdd_handle h) { return h != nullptr && h->magic == 0x6d706464; }

// k-split for a launch of `tiles` output tiles: aim at ~1024 workgroups (four
// per CU) with k-ranges of >= 256, or for a triangle (whose diagonal tiles do
// less work) ~2048 workgroups with k-ranges of >= 512.
int auto_splitk(int64_t tiles, int64_t k, bool tri) {
  const int64_t target = tri ? 2048 : 1024, min_range = tri ? 512 : 256;
  int s = 1;
  while (s < 32 && tiles * s < target && k / (2 * s) >= min_range) s *= 2;
  return s;
}

struct Plan {
  int tile;
  int splitk;
};

Plan choose(const mpdd_handle h, const mpdd_opts* o, int op, bool ta, bool tb, int64_t m,
            int64_t n, int64_t k, bool square_only) {
  Plan pl{-1, 0};
  if (o && o->tile_id >= 0) pl.tile = o->tile_id;
  if (o && o->splitk > 0) pl.splitk = o->splitk;
  if (pl.tile < 0 || pl.splitk == 0) {
    TuneEntry e;
    if (h->tune.lookup(op, ta, tb, m, n, k, e)) {
      if (pl.tile < 0) pl.tile = e.tile;
      if (pl.splitk == 0) pl.splitk = e.splitk;
    }
  }
  if (pl.tile < 0) pl.tile = default_tile(m, n, k, square_only);
  if (pl.splitk == 0) {
    // (a triangle computes only the tiles that meet it)
    const TileInfo* t = tile_info(pl.tile);
    if (!t) return pl;                     // the caller reports the bad tile
    const int64_t tm = (m + t->bm - 1) / t->bm, tn = (n + t->bn - 1) / t->bn;
    const int64_t tiles = square_only ? tm * (tm + 1) / 2 : tm * tn;
    pl.splitk = auto_splitk(tiles, k, square_only);
  }
  return pl;
}

// Caller-provided scratch for the k-split partials (the no-allocation entry
// point): `ptr` holds `bytes` bytes of device memory.
struct FixedScratch {
  void* ptr;
  size_t bytes;
};

int run_plain(mpdd_handle h, const mpdd_opts* o, bool ta, bool tb, int tri, int64_t m, int64_t n,
              int64_t k, mpdd_dd alpha, const double* Ah, const double* Al, int64_t lda,
              const double* Bh, const double* Bl, int64_t ldb, mpdd_dd beta, double* Ch,
              double* Cl, int64_t ldc, hipStream_t st, const FixedScratch* fixed = nullptr) {
  const bool accurate = o && o->algo == MPDD_PLAIN_ACCURATE;
  GemmParams p{};
  p.m = m; p.n = n; p.k = k;
  p.alpha_hi = alpha.hi; p.alpha_lo = alpha.lo;
  p.beta_hi = beta.hi; p.beta_lo = beta.lo;
  p.a_hi = Ah; p.a_lo = Al; p.lda = lda;
  p.b_hi = Bh; p.b_lo = Bl; p.ldb = ldb;
  p.c_hi = Ch; p.c_lo = Cl; p.ldc = ldc;
  p.tri = tri;
  p.beta_zero = is_zero(beta) ? 1 : 0;

  if (is_zero(alpha) || k == 0) return hip_status(launch_scale(p, st));

  const int op = tri ? 1 : 0;
  Plan pl = choose(h, o, op, ta, tb, m, n, k, tri != 0);
  const TileInfo* t = tile_info(pl.tile);
  if (!t) return MPDD_ERR_UNSUPPORTED;
  if (tri && t->bm != t->bn) return MPDD_ERR_UNSUPPORTED;
  if (pl.splitk < 1 || pl.splitk > 64 || (pl.splitk & (pl.splitk - 1)) != 0)
    return MPDD_ERR_UNSUPPORTED;
  p.tiles_m = (int)((m + t->bm - 1) / t->bm);
  p.tiles_n = (int)((n + t->bn - 1) / t->bn);

  int S = pl.splitk;
  // 16 * S * m * n bytes of partials (hi and lo planes)
  auto partial_bytes = [&](int s_) { return 16.0 * s_ * (double)m * (double)n; };
  // a fixed scratch: an automatic split is halved until its partials fit
  // (the result is then that of the same call with opts->splitk = S)
  if (fixed && !(o && o->splitk > 0))
    while (S > 1 && partial_bytes(S) > (double)fixed->bytes) S >>= 1;
  // k-range per slice: a whole number of staged k-tiles
  int64_t chunk = (k + S - 1) / S;
  chunk = (chunk + t->bk - 1) / t->bk * t->bk;
  while (S > 1 && (int64_t)(S - 1) * chunk >= k) S >>= 1;   // no empty slices
  if (S > 1) {
    chunk = (k + S - 1) / S;
    chunk = (chunk + t->bk - 1) / t->bk * t->bk;
  } else {
    chunk = k;
  }
  p.kchunk = chunk;

  if (S == 1) return hip_status(launch_gemm(pl.tile, p, ta, tb, accurate, 1, st));

  const size_t plane = (size_t)S * (size_t)m * (size_t)n * sizeof(double);
  if (fixed) {
    // (an explicit split whose partials do not fit: rejected, nothing enqueued)
    if (partial_bytes(S) > (double)fixed->bytes) return MPDD_ERR_SCRATCH;
    p.w_hi = (double*)fixed->ptr;
    p.w_lo = (double*)((char*)fixed->ptr + plane);
    hipError_t e = launch_gemm(pl.tile, p, ta, tb, accurate, S, st);
    if (e == hipSuccess) e = launch_splitk_reduce(p, S, st);
    return hip_status(e);
  }
  void* w = nullptr;
  if (hipMallocFromPoolAsync(&w, 2 * plane, h->pool, st) != hipSuccess) return MPDD_ERR_ALLOC;
  p.w_hi = (double*)w;
  p.w_lo = (double*)((char*)w + plane);
  hipError_t e = launch_gemm(pl.tile, p, ta, tb, accurate, S, st);
  if (e == hipSuccess) e = launch_splitk_reduce(p, S, st);
  hipError_t ef = hipFreeAsync(w, st);
  if (e != hipSuccess) return MPDD_ERR_HIP;
  return hip_status(ef);
}

}  // namespace

extern "C" {

const char* mpdd_version(void) { return "mpdd 0.1 (gfx950)"; }

size_t mpdd_struct_size(const char* name) {
  if (!name) return 0;
  if (std::strcmp(name, "mpdd_dd") == 0) return sizeof(mpdd_dd);
  if (std::strcmp(name, "mpdd_ddc") == 0) return sizeof(mpdd_ddc);
  if (std::strcmp(name, "mpdd_qd") == 0) return sizeof(mpdd_qd);
  if (std::strcmp(name, "mpdd_opts") == 0) return sizeof(mpdd_opts);
  if (std::strcmp(name, "mpdd_request") == 0) return sizeof(mpdd_request);
  if (std::strcmp(name, "mpdd_timing") == 0) return sizeof(mpdd_timing);
  if (std::strcmp(name, "mpdd_server_stats") == 0) return sizeof(mpdd_server_stats);
  return 0;
}

int mpdd_tile_count(void) { return tile_count(); }

int mpdd_tile_info(int id, int* bm, int* bn, int* bk, int* threads) {
  const TileInfo* t = tile_info(id);
  if (!t) return MPDD_ERR_ARG;
  if (bm) *bm = t->bm;
  if (bn) *bn = t->bn;
  if (bk) *bk = t->bk;
  if (threads) *threads = t->threads;
  return 0;
}

int mpdd_ozaki_digit_widths(int algo, mpdd_int k, int nslices, int* wfirst, int* w) {
  if ((algo != MPDD_OZAKI_I8 && algo != MPDD_OZAKI_F64) || !wfirst || !w || k < 0 ||
      nslices < 1)
    return MPDD_ERR_ARG;
  return ozaki_digit_widths(algo, k, nslices, wfirst, w);
}

int mpdd_ozaki_crt_exponent(mpdd_int k, int nmoduli, int* p) {
  if (!p || k < 0 || nmoduli < 1 || nmoduli > CRT_MAX_MODULI) return MPDD_ERR_ARG;
  if (k > CRT_MAX_K) return MPDD_ERR_UNSUPPORTED;
  const int e = crt_exponent(k, nmoduli);
  if (e == 0) return MPDD_ERR_UNSUPPORTED;
  *p = e;
  return 0;
}

int mpdd_ozaki_split(mpdd_handle h, int algo, const char* trans, mpdd_int rows, mpdd_int k,
                     const double* X_hi, const double* X_lo, mpdd_int ld, int nslices,
                     int* exps, void* slices, mpdd_int ldq, mpdd_int rows_p, void* stream) {
  if (!split_algo(algo)) return MPDD_ERR_ARG;
  const bool nt = lsame(trans, 'N');
  if (!nt && !lsame(trans, 'T') && !lsame(trans, 'C')) return 2;
  if (rows < 0) return 3;
  if (k < 0) return 4;
  if (ld < std::max<mpdd_int>(1, nt ? rows : k)) return 8;
  if (nslices < 1 || nslices > (algo == MPDD_OZAKI_CRT ? CRT_MAX_MODULI : 40)) return 9;
  if (ldq < k || ldq % 64 != 0 || ldq < 64) return 12;
  if (rows_p < rows || rows_p % 64 != 0 || rows_p < 64) return 13;
  if (!handle_ok(h)) return MPDD_ERR_HANDLE;
  if (rows == 0) return 0;
  int wf = 0, w = 0;
  if (algo == MPDD_OZAKI_CRT) {
    if (k > CRT_MAX_K || crt_exponent(k, nslices) == 0) return MPDD_ERR_UNSUPPORTED;
  } else {
    const int e = ozaki_digit_widths(algo, k, nslices, &wf, &w);
    if (e) return e;
  }
  if (!exps || !slices || (k > 0 && (!X_hi || !X_lo))) return MPDD_ERR_ARG;
  return ozaki_split_entry(algo, !nt, rows, k, X_hi, X_lo, ld, nslices, wf, w, exps, slices, ldq,
                           rows_p, (hipStream_t)stream, h->pool);
}

int mpdd_create(mpdd_handle* h, const char* tuner_cache_path) {
  if (!h) return MPDD_ERR_ARG;
  *h = nullptr;
  auto* s = new (std::nothrow) mpdd_handle_s();
  if (!s) return MPDD_ERR_ALLOC;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return MPDD_ERR_HIP;
  }
  // (the device is current: its address of the static scratch)
  if (const int e = static_scratch_init(s->device)) {
    delete s;
    return e;
  }
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = s->device;
  uint64_t keep = UINT64_MAX;
  if (hipMemPoolCreate(&s->pool, &props) != hipSuccess ||
      hipMemPoolSetAttribute(s->pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
    if (s->pool) (void)hipMemPoolDestroy(s->pool);
    delete s;
    return MPDD_ERR_HIP;
  }
  if (tuner_cache_path && tuner_cache_path[0]) {
    if (!s->tune.load(tuner_cache_path)) {
      (void)hipMemPoolDestroy(s->pool);
      delete s;
      return MPDD_ERR_ARG;
    }
  }
  *h = s;
  return 0;
}

int mpdd_destroy(mpdd_handle h) {
  if (!handle_ok(h)) return MPDD_ERR_HANDLE;
  h->magic = 0;
  destroy_stager(h->stager[0]);
  destroy_stager(h->stager[1]);
  // (allocations still being freed on a stream release with their frees)
  (void)hipMemPoolDestroy(h->pool);
  delete h;
  return 0;
}

int mpdd_Rgemm_ex(mpdd_handle h, const mpdd_opts* opts, const char* transa, const char* transb,
                  mpdd_int m, mpdd_int n, mpdd_int k, mpdd_dd alpha, const double* A_hi,
                  const double* A_lo, mpdd_int lda, const double* B_hi, const double* B_lo,
                  mpdd_int ldb, mpdd_dd beta, double* C_hi, double* C_lo, mpdd_int ldc,
                  void* stream) {
  const int info = check_gemm(transa, transb, m, n, k, lda, ldb, ldc);
  if (info) return info;
  if (!handle_ok(h)) return MPDD_ERR_HANDLE;
  const int algo = opts ? opts->algo : MPDD_PLAIN;
  if (algo != MPDD_PLAIN && algo != MPDD_PLAIN_ACCURATE && !split_algo(algo)) return MPDD_ERR_ARG;
  if (m == 0 || n == 0 || ((is_zero(alpha) || k == 0) && is_one(beta))) return 0;
  if (!C_hi || !C_lo) return MPDD_ERR_ARG;
  if (!is_zero(alpha) && k > 0 && (!A_hi || !A_lo || !B_hi || !B_lo)) return MPDD_ERR_ARG;
  const bool ta = !lsame(transa, 'N'), tb = !lsame(transb, 'N');
  hipStream_t st = (hipStream_t)stream;
  if (split_algo(algo))
    return ozaki_gemm(opts, 0, ta, tb, m, n, k, alpha.hi, alpha.lo, A_hi, A_lo, lda, B_hi, B_lo,
                      ldb, beta.hi, beta.lo, C_hi, C_lo, ldc, st, h->pool);
  return run_plain(h, opts, ta, tb, 0, m, n, k, alpha, A_hi, A_lo, lda, B_hi, B_lo, ldb, beta,
                   C_hi, C_lo, ldc, st);
}

int mpdd_Rgemm(mpdd_handle h, const char* transa, const char* transb, mpdd_int m, mpdd_int n,
               mpdd_int k, mpdd_dd alpha, const double* A_hi, const double* A_lo, mpdd_int lda,
               const double* B_hi, const double* B_lo, mpdd_int ldb, mpdd_dd beta,
               double* C_hi, double* C_lo, mpdd_int ldc, void* stream) {
  return mpdd_Rgemm_ex(h, nullptr, transa, transb, m, n, k, alpha, A_hi, A_lo, lda, B_hi, B_lo,
                       ldb, beta, C_hi, C_lo, ldc, stream);
}

int mpdd_Rgemm_noalloc(mpdd_handle h, const mpdd_opts* opts, const char* transa,
                       const char* transb, mpdd_int m, mpdd_int n, mpdd_int k, mpdd_dd alpha,
                       const double* A_hi, const double* A_lo, mpdd_int lda, const double* B_hi,
                       const double* B_lo, mpdd_int ldb, mpdd_dd beta, double* C_hi,
                       double* C_lo, mpdd_int ldc, void* stream) {
  const int info = check_gemm(transa, transb, m, n, k, lda, ldb, ldc);
  if (info) return info;
  if (!handle_ok(h)) return MPDD_ERR_HANDLE;
  const int algo = opts ? opts->algo : MPDD_PLAIN;
  if (split_algo(algo)) return MPDD_ERR_UNSUPPORTED;
  if (algo != MPDD_PLAIN && algo != MPDD_PLAIN_ACCURATE) return MPDD_ERR_ARG;
  if (m == 0 || n == 0 || ((is_zero(alpha) || k == 0) && is_one(beta))) return 0;
  if (!C_hi || !C_lo) return MPDD_ERR_ARG;
  if (!is_zero(alpha) && k > 0 && (!A_hi || !A_lo || !B_hi || !B_lo)) return MPDD_ERR_ARG;
  const FixedScratch fs{static_scratch_ptr(h->device), (size_t)MPDD_STATIC_SCRATCH_BYTES};
  if (!fs.ptr) return MPDD_ERR_HIP;
  const bool ta = !lsame(transa, 'N'), tb = !lsame(transb, 'N');
  return run_plain(h, opts, ta, tb, 0, m, n, k, alpha, A_hi, A_lo, lda, B_hi, B_lo, ldb, beta,
                   C_hi, C_lo, ldc, (hipStream_t)stream, &fs);
}

int mpdd_Rsyrk_ex(mpdd_handle h, const mpdd_opts* opts, const char* uplo, const char* trans,
                  mpdd_int n, mpdd_int k, mpdd_dd alpha, const double* A_hi,
                  const double* A_lo, mpdd_int lda, mpdd_dd beta, double* C_hi,
                  double* C_lo, mpdd_int ldc, void* stream) {
  const int info = check_syrk(uplo, trans, n, k, lda, ldc);
  if (info) return info;
  if (!handle_ok(h)) return MPDD_ERR_HANDLE;
  const int algo = opts ? opts->algo : MPDD_PLAIN;
  if (algo != MPDD_PLAIN && algo != MPDD_PLAIN_ACCURATE && !split_algo(algo)) return MPDD_ERR_ARG;
  if (n == 0 || ((is_zero(alpha) || k == 0) && is_one(beta))) return 0;
  if (!C_hi || !C_lo) return MPDD_ERR_ARG;
  if (!is_zero(alpha) && k > 0 && (!A_hi || !A_lo)) return MPDD_ERR_ARG;
  // trans N: op(A) = A (n x k), op(B) = A^T; trans T: op(A) = A^T, op(B) = A.
  const bool ta = !lsame(trans, 'N');
  const bool tb = !ta;
  const int tri = lsame(uplo, 'U') ? 1 : 2;
  if (split_algo(algo))
    return ozaki_gemm(opts, tri, ta, tb, n, n, k, alpha.hi, alpha.lo, A_hi, A_lo, lda, A_hi,
                      A_lo, lda, beta.hi, beta.lo, C_hi, C_lo, ldc, (hipStream_t)stream, h->pool);
  return run_plain(h, opts, ta, tb, tri, n, n, k, alpha, A_hi, A_lo, lda, A_hi, A_lo, lda, beta,
                   C_hi, C_lo, ldc, (hipStream_t)stream);
}

// Cgemm.  With sA = -1 when op(A) conjugates (transa 'C'), else +1, and
// op_r(A), op_i(A) the real transposition of the real and imaginary planes:
//  4M (default):
//   Re P = op_r(Ar) op_r(Br) - sA sB op_r(Ai) op_r(Bi)
//   Im P = sB op_r(Ar) op_r(Bi) + sA op_r(Ai) op_r(Br),
//   four plain dd products (the second of each pair accumulates onto the first
//   through beta = 1);
//  3M (MPDD_COMPLEX_3M): with R1 = op_r(Ar) op_r(Br), R2 = sA sB op_r(Ai) op_r(Bi)
//   and R3 = op_r(Ar + sA Ai) op_r(Br + sB Bi) (the sums formed in dd,
//   elementwise, into scratch), Re P = R1 - R2 and Im P = R3 - R1 - R2: three
//   products, a quarter less arithmetic, at the price of the cancellation in
//   Im P (its error is relative to |Ar + Ai| |Br + Bi| rather than to |P|);
// then C <- alpha P + beta C in complex dd.
int mpdd_Cgemm_ex(mpdd_handle h, const mpdd_opts* opts, const char* transa, const char* transb,
                  mpdd_int m, mpdd_int n, mpdd_int k, mpdd_ddc alpha, const double* A_re_hi,
                  const double* A_re_lo, const double* A_im_hi, const double* A_im_lo,
                  mpdd_int lda, const double* B_re_hi, const double* B_re_lo,
                  const double* B_im_hi, const double* B_im_lo, mpdd_int ldb, mpdd_ddc beta,
                  double* C_re_hi, double* C_re_lo, double* C_im_hi, double* C_im_lo,
                  mpdd_int ldc, void* stream) {
  const int info = check_gemm(transa, transb, m, n, k, lda, ldb, ldc);
  if (info) return info;
  if (!handle_ok(h)) return MPDD_ERR_HANDLE;
  const int algo = opts ? opts->algo : MPDD_PLAIN;
  if (algo != MPDD_PLAIN && algo != MPDD_COMPLEX_3M && !split_algo(algo)) return MPDD_ERR_ARG;
  const bool split = split_algo(algo);
  const bool alpha_zero = is_zero(alpha.re) && is_zero(alpha.im);
  const bool beta_zero = is_zero(beta.re) && is_zero(beta.im);
  const bool beta_one = is_one(beta.re) && is_zero(beta.im);
  if (m == 0 || n == 0 || ((alpha_zero || k == 0) && beta_one)) return 0;
  if (!C_re_hi || !C_re_lo || !C_im_hi || !C_im_lo) return MPDD_ERR_ARG;
  const bool use_p = !alpha_zero && k > 0;
  if (use_p && (!A_re_hi || !A_re_lo || !A_im_hi || !A_im_lo || !B_re_hi || !B_re_lo ||
                !B_im_hi || !B_im_lo))
    return MPDD_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  CEpilogue e{};
  e.m = m; e.n = n;
  e.alpha[0] = alpha.re.hi; e.alpha[1] = alpha.re.lo;
  e.alpha[2] = alpha.im.hi; e.alpha[3] = alpha.im.lo;
  e.beta[0] = beta.re.hi; e.beta[1] = beta.re.lo;
  e.beta[2] = beta.im.hi; e.beta[3] = beta.im.lo;
  e.c_rh = C_re_hi; e.c_rl = C_re_lo; e.c_ih = C_im_hi; e.c_il = C_im_lo;
  e.ldc = ldc;
  e.beta_zero = beta_zero ? 1 : 0;
  e.use_p = use_p ? 1 : 0;
  if (!use_p) return hip_status(launch_cgemm_epilogue(e, st));

  // the real products use the caller's tile / k-split choice
  mpdd_opts ro{MPDD_PLAIN, 0, opts ? opts->tile_id : -1, opts ? opts->splitk : 0};
  const bool ta = !lsame(transa, 'N'), tb = !lsame(transb, 'N');
  const double sa = lsame(transa, 'C') ? -1.0 : 1.0, sb = lsame(transb, 'C') ? -1.0 : 1.0;
  const size_t plane = (size_t)m * (size_t)n * sizeof(double);
  const mpdd_dd zero{0.0, 0.0}, one{1.0, 0.0};
  e.ldp = m;
  if (algo == MPDD_OZAKI_CRT) {
    // modular form: the complex product from three residue products per
    // modulus, exact in integers, into P; then the same complex epilogue
    void* w = nullptr;
    if (hipMallocFromPoolAsync(&w, 4 * plane, h->pool, st) != hipSuccess) return MPDD_ERR_ALLOC;
    double* pp[4];
    for (int q = 0; q < 4; ++q) pp[q] = (double*)((char*)w + q * plane);
    const int opa = !ta ? 0 : lsame(transa, 'C') ? 2 : 1;
    const int opb = !tb ? 0 : lsame(transb, 'C') ? 2 : 1;
    const double* av[4] = {A_re_hi, A_re_lo, A_im_hi, A_im_lo};
    const double* bv[4] = {B_re_hi, B_re_lo, B_im_hi, B_im_lo};
    int rc = ozaki_crt_cgemm(opts, opa, opb, m, n, k, av, lda, bv, ldb, pp[0], pp[1], pp[2],
                             pp[3], st, h->pool);
    if (!rc) {
      e.p_rh = pp[0]; e.p_rl = pp[1]; e.p_ih = pp[2]; e.p_il = pp[3];
      rc = hip_status(launch_cgemm_epilogue(e, st));
    }
    const hipError_t ef = hipFreeAsync(w, st);
    if (rc) return rc;
    return hip_status(ef);
  }
  if (algo != MPDD_COMPLEX_3M) {
    // four real products (plain, or split form: each an Rgemm_ex of the
    // caller's split algo, slice count and INT8 tiling)
    auto product = [&](mpdd_dd a, const double* xh, const double* xl, const double* yh,
                       const double* yl, mpdd_dd b, double* ph, double* pl) -> int {
      if (split)
        return ozaki_gemm(opts, 0, ta, tb, m, n, k, a.hi, a.lo, xh, xl, lda, yh, yl, ldb, b.hi,
                          b.lo, ph, pl, m, st, h->pool);
      return run_plain(h, &ro, ta, tb, 0, m, n, k, a, xh, xl, lda, yh, yl, ldb, b, ph, pl, m, st);
    };
    void* w = nullptr;
    if (hipMallocFromPoolAsync(&w, 4 * plane, h->pool, st) != hipSuccess) return MPDD_ERR_ALLOC;
    double* prh = (double*)w;
    double* prl = (double*)((char*)w + plane);
    double* pih = (double*)((char*)w + 2 * plane);
    double* pil = (double*)((char*)w + 3 * plane);
    int rc = product(one, A_re_hi, A_re_lo, B_re_hi, B_re_lo, zero, prh, prl);
    if (!rc)
      rc = product(mpdd_dd{-sa * sb, 0.0}, A_im_hi, A_im_lo, B_im_hi, B_im_lo, one, prh, prl);
    if (!rc) rc = product(mpdd_dd{sb, 0.0}, A_re_hi, A_re_lo, B_im_hi, B_im_lo, zero, pih, pil);
    if (!rc) rc = product(mpdd_dd{sa, 0.0}, A_im_hi, A_im_lo, B_re_hi, B_re_lo, one, pih, pil);
    if (!rc) {
      e.p_rh = prh; e.p_rl = prl; e.p_ih = pih; e.p_il = pil;
      rc = hip_status(launch_cgemm_epilogue(e, st));
    }
    const hipError_t ef = hipFreeAsync(w, st);
    if (rc) return rc;
    return hip_status(ef);
  }
  // 3M: the operand sums in compact storage (op(A): rows_a x cols_a as stored)
  const int64_t ra = ta ? k : m, ca = ta ? m : k, rb = tb ? n : k, cb = tb ? k : n;
  const size_t sa_bytes = (size_t)ra * ca * sizeof(double), sb_bytes = (size_t)rb * cb * sizeof(double);
  void* w = nullptr;
  if (hipMallocFromPoolAsync(&w, 6 * plane + 2 * sa_bytes + 2 * sb_bytes, h->pool, st) !=
      hipSuccess)
    return MPDD_ERR_ALLOC;
  char* base = (char*)w;
  double* r1h = (double*)base;
  double* r1l = (double*)(base + plane);
  double* r2h = (double*)(base + 2 * plane);
  double* r2l = (double*)(base + 3 * plane);
  double* r3h = (double*)(base + 4 * plane);
  double* r3l = (double*)(base + 5 * plane);
  double* sah = (double*)(base + 6 * plane);
  double* sal = (double*)(base + 6 * plane + sa_bytes);
  double* sbh = (double*)(base + 6 * plane + 2 * sa_bytes);
  double* sbl = (double*)(base + 6 * plane + 2 * sa_bytes + sb_bytes);
  int rc = hip_status(launch_dd_axpy_planes(A_re_hi, A_re_lo, A_im_hi, A_im_lo, lda, sa, ra, ca,
                                            sah, sal, st));
  if (!rc)
    rc = hip_status(launch_dd_axpy_planes(B_re_hi, B_re_lo, B_im_hi, B_im_lo, ldb, sb, rb, cb,
                                          sbh, sbl, st));
  if (!rc)
    rc = run_plain(h, &ro, ta, tb, 0, m, n, k, one, A_re_hi, A_re_lo, lda, B_re_hi, B_re_lo, ldb,
                   zero, r1h, r1l, m, st);
  if (!rc)
    rc = run_plain(h, &ro, ta, tb, 0, m, n, k, mpdd_dd{sa * sb, 0.0}, A_im_hi, A_im_lo, lda,
                   B_im_hi, B_im_lo, ldb, zero, r2h, r2l, m, st);
  if (!rc)
    rc = run_plain(h, &ro, ta, tb, 0, m, n, k, one, sah, sal, ra, sbh, sbl, rb, zero, r3h, r3l, m,
                   st);
  if (!rc) {
    e.p_rh = r1h; e.p_rl = r1l; e.p_ih = r2h; e.p_il = r2l;
    e.q_h = r3h; e.q_l = r3l;
    e.three_m = 1;
    rc = hip_status(launch_cgemm_epilogue(e, st));
  }
  const hipError_t ef = hipFreeAsync(w, st);
  if (rc) return rc;
  return hip_status(ef);
}

int mpdd_Cgemm(mpdd_handle h, const char* transa, const char* transb, mpdd_int m, mpdd_int n,
               mpdd_int k, mpdd_ddc alpha, const double* A_re_hi, const double* A_re_lo,
               const double* A_im_hi, const double* A_im_lo, mpdd_int lda,
               const double* B_re_hi, const double* B_re_lo, const double* B_im_hi,
               const double* B_im_lo, mpdd_int ldb, mpdd_ddc beta, double* C_re_hi,
               double* C_re_lo, double* C_im_hi, double* C_im_lo, mpdd_int ldc, void* stream) {
  return mpdd_Cgemm_ex(h, nullptr, transa, transb, m, n, k, alpha, A_re_hi, A_re_lo, A_im_hi,
                       A_im_lo, lda, B_re_hi, B_re_lo, B_im_hi, B_im_lo, ldb, beta, C_re_hi,
                       C_re_lo, C_im_hi, C_im_lo, ldc, stream);
}

// Rpotrf, blocked (LAPACK DPOTRF's left-looking order, with look-ahead).
// Block b (columns j = b*nb .. j+jb; 'L' shown, 'U' is the transpose) needs
// its block column A(j:n, j:j+jb), copied to a scratch P_b, minus the
// contributions of every factored block column c < b.  Those are applied in
// two products: all c < b-1 at once (the bulk, on one of two bulk streams,
// started as soon as block b-2 is finished, so it overlaps the critical work
// of block b-1), then c = b-1 alone (k = nb, on the caller's stream).  Then
// the block kernel factors P_b's diagonal block into A and inverts the factor
// (W), and the rest of P_b is multiplied by W^T into A.  P has three buffers;
// events order the three streams.  The diagonal block rides along in every product
// (both of its triangles computed in P), so A's opposite triangle is never
// written.  The first failing pivot is recorded in a device word that later
// block kernels respect (they return at once); the host reads it every
// POTRF_CHECK blocks and at the end, and stops launching once it is set.
// After a failure, the columns before the failing block hold the factor and
// A(k,k) the pivot; later columns are unspecified.
// One blocked Cholesky in progress: the streams, events and scratch of the
// left-looking schedule with look-ahead, kept for every panel of a call.
//
// Bulk updates alternate between two streams, so that one block's bulk
// product can start while the previous block's is still running; block b
// keeps its column in P[b % NP], so the bulk update of block b may start as
// soon as block b-2 is finished while blocks b-1 and b-2 still hold theirs.
struct PotrfRun {
  static constexpr int NP = 3;
  static constexpr int64_t CHECK = 16;   // blocks between host reads of the failure word
  mpdd_handle h = nullptr;
  bool upper = false;
  int64_t lda = 0, nb = 0;
  hipStream_t st = nullptr;
  hipStream_t sb[2] = {nullptr, nullptr};
  hipEvent_t ev_bulk[NP] = {}, ev_done[NP] = {};
  hipEvent_t ev_start = nullptr, ev_end[2] = {nullptr, nullptr};
  void* ws = nullptr;
  double *w_hi = nullptr, *w_lo = nullptr;
  double* p_hi[NP] = {};
  double* p_lo[NP] = {};
  long long* d_info = nullptr;
  long long hinfo = 0;       // the failure word as last read by the host
  bool joined = true;        // the bulk streams' work is ordered before st's

  // Streams, events and scratch for matrices of order <= n (W: nb x nb, the
  // block-column copies P: n x nb, two planes each); the failure word is
  // cleared on st.
  int open(mpdd_handle h_, bool upper_, int64_t n, int64_t lda_, int64_t nb_, hipStream_t st_) {
    h = h_;
    upper = upper_;
    lda = lda_;
    nb = nb_;
    st = st_;
    auto make_event = [](hipEvent_t& e) {
      return hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    };
    bool ok = true;
    for (int t = 0; t < 2 && ok; ++t)
      ok = hipStreamCreateWithFlags(&sb[t], hipStreamNonBlocking) == hipSuccess;
    for (int t = 0; t < NP && ok; ++t) ok = make_event(ev_bulk[t]) && make_event(ev_done[t]);
    ok = ok && make_event(ev_start) && make_event(ev_end[0]) && make_event(ev_end[1]);
    if (!ok) return MPDD_ERR_HIP;
    const size_t wb = (size_t)nb * nb * sizeof(double);
    const size_t pb = (size_t)n * nb * sizeof(double);
    if (hipMallocFromPoolAsync(&ws, 2 * wb + 2 * NP * pb + 256, h->pool, st) != hipSuccess) {
      ws = nullptr;
      return MPDD_ERR_ALLOC;
    }
    w_hi = (double*)ws;
    w_lo = (double*)((char*)ws + wb);
    for (int t = 0; t < NP; ++t) {
      p_hi[t] = (double*)((char*)ws + 2 * wb + 2 * t * pb);
      p_lo[t] = (double*)((char*)ws + 2 * wb + (2 * t + 1) * pb);
    }
    d_info = (long long*)((char*)ws + 2 * wb + 2 * NP * pb);
    return hipMemsetAsync(d_info, 0, sizeof(long long), st) == hipSuccess ? 0 : MPDD_ERR_HIP;
  }

  // Enqueue the factorisation of the first ncols columns (upper: rows) of the
  // n x n matrix A (n no larger than open's), uplo triangle, on st: a failing
  // pivot is recorded as its column + col0 + 1 in the failure word, and later
  // block kernels leave their blocks alone.  With ncols = n this is the whole
  // factorisation; with fewer, the factored columns are a panel of a
  // right-looking factorisation, whose trailing matrix has received the
  // updates of the panels before it.  The bulk streams start after the work
  // already on st and are joined back into st at the end.  With `checks`,
  // the host reads the failure word every CHECK blocks and stops at a
  // failure (synchronising st); without, nothing waits on the host.
  int factor(double* A_hi, double* A_lo, int64_t n, int64_t ncols, int64_t col0, bool checks) {
    int rc = 0;
    if (hipEventRecord(ev_start, st) != hipSuccess ||
        hipStreamWaitEvent(sb[0], ev_start, 0) != hipSuccess ||
        hipStreamWaitEvent(sb[1], ev_start, 0) != hipSuccess)
      return MPDD_ERR_HIP;
    const mpdd_dd one{1.0, 0.0}, mone{-1.0, 0.0}, zero{0.0, 0.0};
    // the panel solve is a skinny product with k = jb: 32 x 32 tiles give the
    // CUs more workgroups
    mpdd_opts small{MPDD_PLAIN, 0, 2, 1};
    auto at = [&](double* base, int64_t i, int64_t j) { return base + i + j * lda; };
    const int64_t nblk = (ncols + nb - 1) / nb;
    // copy block column b into P[b % NP] on stream s
    auto load_block = [&](int64_t b, hipStream_t s) -> int {
      const int64_t j = b * nb, jb = std::min<int64_t>(nb, ncols - j), rows = n - j;
      const int64_t ldp = upper ? jb : rows;
      const int64_t w = upper ? jb : rows, hgt = upper ? rows : jb;
      for (int t = 0; t < 2; ++t) {
        double* dst = t ? p_lo[b % NP] : p_hi[b % NP];
        const double* src = t ? at(A_lo, j, j) : at(A_hi, j, j);
        if (hipMemcpy2DAsync(dst, ldp * sizeof(double), src, lda * sizeof(double),
                             w * sizeof(double), hgt, hipMemcpyDeviceToDevice, s) != hipSuccess)
          return MPDD_ERR_HIP;
      }
      return 0;
    };
    // P[b % NP] -= contributions of block columns [c0, c1) (c1 > c0) on stream s
    auto update_block = [&](int64_t b, int64_t c0, int64_t c1, hipStream_t s) -> int {
      const int64_t j = b * nb, jb = std::min<int64_t>(nb, ncols - j), rows = n - j;
      const int64_t k0 = c0 * nb, kk = c1 * nb - k0;
      double* ph = p_hi[b % NP];
      double* pl = p_lo[b % NP];
      if (!upper)
        return run_plain(h, nullptr, false, true, 0, rows, jb, kk, mone, at(A_hi, j, k0),
                         at(A_lo, j, k0), lda, at(A_hi, j, k0), at(A_lo, j, k0), lda, one, ph,
                         pl, rows, s);
      return run_plain(h, nullptr, true, false, 0, jb, rows, kk, mone, at(A_hi, k0, j),
                       at(A_lo, k0, j), lda, at(A_hi, k0, j), at(A_lo, k0, j), lda, one, ph, pl,
                       jb, s);
    };
    // bulk stream t & 1, block t: load P_t and apply block columns [0, t-1),
    // once block t-2 is finished (which also frees P[t % NP], last used by
    // block t-3)
    auto bulk = [&](int64_t t) -> int {
      hipStream_t s = sb[t & 1];
      if (t >= 2 && hipStreamWaitEvent(s, ev_done[(t - 2) % NP], 0) != hipSuccess)
        return MPDD_ERR_HIP;
      int r = load_block(t, s);
      if (!r && t >= 2) r = update_block(t, 0, t - 1, s);
      if (!r && hipEventRecord(ev_bulk[t % NP], s) != hipSuccess) r = MPDD_ERR_HIP;
      return r;
    };
    joined = false;
    rc = bulk(0);
    if (!rc && nblk > 1) rc = bulk(1);
    for (int64_t b = 0; b < nblk && !rc; ++b) {
      const int64_t j = b * nb, jb = std::min<int64_t>(nb, ncols - j), rows = n - j;
      const int64_t ldp = upper ? jb : rows;
      // critical path of block b on the caller's stream
      if (hipStreamWaitEvent(st, ev_bulk[b % NP], 0) != hipSuccess) {
        rc = MPDD_ERR_HIP;
        break;
      }
      if (b >= 1 && (rc = update_block(b, b - 1, b, st)) != 0) break;
      if (launch_potf2_block(p_hi[b % NP], p_lo[b % NP], ldp, at(A_hi, j, j), at(A_lo, j, j),
                             lda, (int)jb, upper ? 1 : 0, w_hi, w_lo, d_info,
                             (long long)(col0 + j), st) != hipSuccess) {
        rc = MPDD_ERR_HIP;
        break;
      }
      if (rows > jb) {
        // panel solve: lower A(j+jb:n, j:j+jb) = P(jb:, :) W^T; upper
        // A(j:j+jb, j+jb:n) = W P(:, jb:)   (W = U^-T in the lower view)
        if (!upper)
          rc = run_plain(h, &small, false, true, 0, rows - jb, jb, jb, one, p_hi[b % NP] + jb,
                         p_lo[b % NP] + jb, ldp, w_hi, w_lo, jb, zero, at(A_hi, j + jb, j),
                         at(A_lo, j + jb, j), lda, st);
        else
          rc = run_plain(h, &small, false, false, 0, jb, rows - jb, jb, one, w_hi, w_lo, jb,
                         p_hi[b % NP] + jb * jb, p_lo[b % NP] + jb * jb, ldp, zero,
                         at(A_hi, j, j + jb), at(A_lo, j, j + jb), lda, st);
        if (rc) break;
      }
      // block b finished: block b+2's bulk update may start
      if (hipEventRecord(ev_done[b % NP], st) != hipSuccess) {
        rc = MPDD_ERR_HIP;
        break;
      }
      if (b + 2 < nblk && (rc = bulk(b + 2)) != 0) break;
      // every CHECK blocks: stop once a pivot has failed
      if (checks && b % CHECK == CHECK - 1) {
        if (hipMemcpyAsync(&hinfo, d_info, sizeof(long long), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
          rc = MPDD_ERR_HIP;
          break;
        }
        if (hinfo) break;
      }
    }
    // st waits for the bulk streams (later work on st, and the release of
    // the scratch, come after them)
    bool ok = true;
    for (int t = 0; t < 2; ++t)
      ok = ok && hipEventRecord(ev_end[t], sb[t]) == hipSuccess &&
           hipStreamWaitEvent(st, ev_end[t], 0) == hipSuccess;
    joined = ok;
    if (!rc && !ok) rc = MPDD_ERR_HIP;
    return rc;
  }

  // Read the failure word (unless rc != 0 or a failure has been read),
  // free the scratch, wait for st and release the streams and events.
  // Returns rc, or the first error of these steps.
  int close(int rc) {
    if (ws && !rc && !hinfo &&
        (hipMemcpyAsync(&hinfo, d_info, sizeof(long long), hipMemcpyDeviceToHost, st) !=
             hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess))
      rc = MPDD_ERR_HIP;
    if (!joined)
      for (int t = 0; t < 2; ++t)
        if (sb[t]) (void)hipStreamSynchronize(sb[t]);
    const hipError_t ef = ws ? hipFreeAsync(ws, st) : hipSuccess;
    const hipError_t es = hipStreamSynchronize(st);
    for (int t = 0; t < NP; ++t) {
      if (ev_bulk[t]) (void)hipEventDestroy(ev_bulk[t]);
      if (ev_done[t]) (void)hipEventDestroy(ev_done[t]);
    }
    if (ev_start) (void)hipEventDestroy(ev_start);
    for (int t = 0; t < 2; ++t) {
      if (ev_end[t]) (void)hipEventDestroy(ev_end[t]);
      if (sb[t]) (void)hipStreamDestroy(sb[t]);
    }
    if (rc) return rc;
    return (ef != hipSuccess || es != hipSuccess) ? MPDD_ERR_HIP : 0;
  }
};

int mpdd_Rpotrf_nb(mpdd_handle h, const char* uplo, mpdd_int n, double* A_hi, double* A_lo,
                   mpdd_int lda, mpdd_int nb, mpdd_int* info, void* stream) {
  return mpdd_Rpotrf_ex(h, nullptr, uplo, n, A_hi, A_lo, lda, nb, info, stream);
}

// Panel width of the right-looking form (split-form trailing updates), in
// columns, rounded down to whole blocks (measured at n = 8192 with nb = 64:
// 1024 against 512 and 2048).  A compile-time knob for measurements.
#ifndef MPDD_POTRF_PANEL_COLUMNS
#define MPDD_POTRF_PANEL_COLUMNS 1024
#endif
constexpr int64_t POTRF_PANEL_COLUMNS = MPDD_POTRF_PANEL_COLUMNS;

int mpdd_Rpotrf_ex(mpdd_handle h, const mpdd_opts* opts, const char* uplo, mpdd_int n,
                   double* A_hi, double* A_lo, mpdd_int lda, mpdd_int nb, mpdd_int* info,
                   void* stream) {
  if (!info) return MPDD_ERR_ARG;
  *info = 0;
  const bool upper = lsame(uplo, 'U');
  if (!upper && !lsame(uplo, 'L')) { *info = -1; return 0; }
  if (n < 0) { *info = -2; return 0; }
  if (lda < std::max<mpdd_int>(1, n)) { *info = -4; return 0; }
  if (!handle_ok(h)) return MPDD_ERR_HANDLE;
  const int algo = opts ? opts->algo : MPDD_PLAIN;
  if (algo != MPDD_PLAIN && !split_algo(algo)) return MPDD_ERR_ARG;
  if (nb == 0) nb = 64;
  if (nb < 1 || nb > 64) return MPDD_ERR_UNSUPPORTED;
  if (n == 0) return 0;
  if (!A_hi || !A_lo) return MPDD_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  PotrfRun run;
  int rc = run.open(h, upper, n, lda, nb, st);
  if (!rc && algo == MPDD_PLAIN) {
    rc = run.factor(A_hi, A_lo, n, n, 0, true);
  } else if (!rc) {
    // Right-looking over panels of POTRF_PANEL_COLUMNS columns: the panel's
    // columns (rows for 'U') are factored left-looking inside the trailing
    // matrix, then the rest of the trailing matrix takes the panel's update
    // in one split-form Rsyrk: lower A22 -= L21 L21^T, upper A22 -= U12^T U12.
    // Everything is enqueued on st without host round trips; a failing pivot
    // stays recorded in the failure word, read at the end (the factor beyond
    // it is unspecified, as for the plain form).
    const int64_t pw = std::max<int64_t>(1, POTRF_PANEL_COLUMNS / nb) * nb;
    const mpdd_opts so{algo, opts->nslices, -1, 0};
    const mpdd_dd one{1.0, 0.0}, mone{-1.0, 0.0};
    for (int64_t j0 = 0; j0 < n && !rc; j0 += pw) {
      const int64_t rest = n - j0, w = std::min(pw, rest);
      double* ah = A_hi + j0 + j0 * lda;
      double* al = A_lo + j0 + j0 * lda;
      rc = run.factor(ah, al, rest, w, j0, false);
      if (!rc && rest > w) {
        const int64_t off = upper ? w * lda : w;      // U12 or L21
        rc = mpdd_Rsyrk_ex(h, &so, upper ? "U" : "L", upper ? "T" : "N", rest - w, w, mone,
                           ah + off, al + off, lda, one, ah + w + w * lda, al + w + w * lda,
                           lda, stream);
      }
    }
  }
  rc = run.close(rc);
  if (rc) return rc;
  *info = (mpdd_int)run.hinfo;
  return 0;
}

int mpdd_Rpotrf(mpdd_handle h, const char* uplo, mpdd_int n, double* A_hi, double* A_lo,
                mpdd_int lda, mpdd_int* info, void* stream) {
  return mpdd_Rpotrf_nb(h, uplo, n, A_hi, A_lo, lda, 0, info, stream);
}

// Quad-double Rgemm: one launch of the qd tile kernel (or the scale kernel
// when alpha = 0 or k = 0).
int mpdd_Qgemm(mpdd_handle h, const char* transa, const char* transb, mpdd_int m, mpdd_int n,
               mpdd_int k, mpdd_qd alpha, const double* A0, const double* A1, const double* A2,
               const double* A3, mpdd_int lda, const double* B0, const double* B1,
               const double* B2, const double* B3, mpdd_int ldb, mpdd_qd beta, double* C0,
               double* C1, double* C2, double* C3, mpdd_int ldc, void* stream) {
  return mpdd_Qgemm_ex(h, nullptr, transa, transb, m, n, k, alpha, A0, A1, A2, A3, lda, B0, B1,
                       B2, B3, ldb, beta, C0, C1, C2, C3, ldc, stream);
}

int mpdd_Qgemm_ex(mpdd_handle h, const mpdd_opts* opts, const char* transa, const char* transb,
                  mpdd_int m, mpdd_int n, mpdd_int k, mpdd_qd alpha, const double* A0,
                  const double* A1, const double* A2, const double* A3, mpdd_int lda,
                  const double* B0, const double* B1, const double* B2, const double* B3,
                  mpdd_int ldb, mpdd_qd beta, double* C0, double* C1, double* C2, double* C3,
                  mpdd_int ldc, void* stream) {
  const int info = check_gemm(transa, transb, m, n, k, lda, ldb, ldc);
  if (info) return info;
  if (!handle_ok(h)) return MPDD_ERR_HANDLE;
  const int algo = opts ? opts->algo : MPDD_PLAIN;
  if (algo != MPDD_PLAIN && algo != MPDD_OZAKI_I8 && algo != MPDD_OZAKI_CRT) return MPDD_ERR_ARG;
  auto qzero = [](const mpdd_qd& x) { return x.x[0] == 0 && x.x[1] == 0 && x.x[2] == 0 && x.x[3] == 0; };
  const bool alpha_zero = qzero(alpha), beta_zero = qzero(beta);
  const bool beta_one = beta.x[0] == 1.0 && beta.x[1] == 0 && beta.x[2] == 0 && beta.x[3] == 0;
  if (m == 0 || n == 0 || ((alpha_zero || k == 0) && beta_one)) return 0;
  if (!C0 || !C1 || !C2 || !C3) return MPDD_ERR_ARG;
  const bool use_ab = !alpha_zero && k > 0;
  if (use_ab && (!A0 || !A1 || !A2 || !A3 || !B0 || !B1 || !B2 || !B3)) return MPDD_ERR_ARG;
  QgemmParams p{};
  p.m = m; p.n = n; p.k = k;
  for (int t = 0; t < 4; ++t) {
    p.alpha[t] = alpha.x[t];
    p.beta[t] = beta.x[t];
  }
  p.a[0] = A0; p.a[1] = A1; p.a[2] = A2; p.a[3] = A3; p.lda = lda;
  p.b[0] = B0; p.b[1] = B1; p.b[2] = B2; p.b[3] = B3; p.ldb = ldb;
  p.c[0] = C0; p.c[1] = C1; p.c[2] = C2; p.c[3] = C3; p.ldc = ldc;
  p.beta_zero = beta_zero ? 1 : 0;
  p.scale_only = use_ab ? 0 : 1;
  if (algo == MPDD_OZAKI_CRT && use_ab)
    return ozaki_crt_qgemm(opts, !lsame(transa, 'N'), !lsame(transb, 'N'), m, n, k, p.alpha,
                           p.a, lda, p.b, ldb, p.beta, p.beta_zero, p.c, ldc,
                           (hipStream_t)stream, h->pool);
  if (algo == MPDD_OZAKI_I8 && use_ab)
    return ozaki_qgemm(opts, !lsame(transa, 'N'), !lsame(transb, 'N'), m, n, k, p.alpha, p.a,
                       lda, p.b, ldb, p.beta, p.beta_zero, p.c, ldc, (hipStream_t)stream,
                       h->pool);
  return hip_status(launch_qgemm(p, !lsame(transa, 'N'), !lsame(transb, 'N'),
                                 (hipStream_t)stream));
}

int mpdd_Rsyrk(mpdd_handle h, const char* uplo, const char* trans, mpdd_int n, mpdd_int k,
               mpdd_dd alpha, const double* A_hi, const double* A_lo, mpdd_int lda,
               mpdd_dd beta, double* C_hi, double* C_lo, mpdd_int ldc, void* stream) {
  return mpdd_Rsyrk_ex(h, nullptr, uplo, trans, n, k, alpha, A_hi, A_lo, lda, beta, C_hi, C_lo,
                       ldc, stream);
}

}  // extern "C"

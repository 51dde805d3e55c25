/*
 * mpdd.h -- C ABI of libmpdd: double-double (dd) Rgemm and Rsyrk on one AMD
 * Instinct MI355X (gfx950).
 *
 * Operations (MPLAPACK 2.0.1 manual, section "How to use reference MPBLAS",
 * which gives Rgemm the calling convention of BLAS DGEMM, and Table
 * "mpblasroutines", which lists Rgemm and Rsyrk among the level-3 MPBLAS
 * routines; the CUDA dd versions of both are the manual's section "CUDA
 * accelerated MPBLAS"):
 *
 *   Rgemm:  C <- alpha * op(A) * op(B) + beta * C,  op(X) = X or X^T
 *   Rsyrk:  C <- alpha * A * A^T + beta * C   (trans = "N")
 *           C <- alpha * A^T * A + beta * C   (trans = "T" or "C")
 *           updating only the uplo triangle of C, diagonal included.
 *
 * Number format (section "Supported Floating point formats"): a dd value is
 * the unevaluated sum hi + lo of two binary64 numbers, |lo| <= ulp(hi)/2,
 * about 106 significant bits (Table "rlamch_dd": epsilon 2^-104).
 *
 * Storage.  Every matrix is column-major with a leading dimension, as in
 * MPBLAS (entry (i, j) of X lives at X[i + j*ldx], 0-based), and is held as
 * TWO separate binary64 planes of identical layout: X_hi and X_lo.  All matrix
 * pointers are DEVICE pointers (hipMalloc / torch allocations on the current
 * device).  Rows ld..: the padding rows between the matrix's row count and
 * its leading dimension are never read or written.  Scalars alpha and beta are
 * normalised dd values passed by value.
 *
 * Flags.  Only the first character counts and case is ignored (MPBLAS
 * Mlsame): trans in {N, T, C} (C means T for real data), uplo in {U, L}.
 *
 * Return value ("info"):
 *   0   success (work enqueued on `stream`; the call does not wait for it);
 *  >0   the 1-based position of the first invalid argument, numbered as in
 *       the BLAS argument lists (Rgemm: 1 transa, 2 transb, 3 m, 4 n, 5 k,
 *       8 lda, 10 ldb, 13 ldc; Rsyrk: 1 uplo, 2 trans, 3 n, 4 k, 7 lda,
 *       10 ldc) -- the codes BLAS xerbla reports, as the manual's MPBLAS
 *       quality-assurance section requires.  Nothing is enqueued and C is
 *       untouched.  The library never prints or aborts.
 *  <0   a runtime error, one of the MPDD_ERR_* codes below.
 *
 * Semantics as BLAS: quick return (C untouched) when m = 0 or n = 0, or when
 * (alpha = 0 or k = 0) and beta = 1.  When alpha = 0 or k = 0, A and B are not
 * read and may be NULL.  When beta = 0, C is written without being read (NaN
 * in C does not propagate).  Rsyrk never reads or writes the opposite
 * triangle.
 *
 * Ownership and asynchrony.  The caller owns A, B and C; they must stay valid
 * until the work enqueued on `stream` has completed.  `stream` is a
 * hipStream_t passed as void* (NULL = the legacy default stream).  The handle
 * belongs to the device current at mpdd_create and owns a tuning table and a
 * stream-ordered memory pool on that device: scratch memory that a call
 * needs (split-k partial sums, split-form slices, ...) is allocated from the
 * pool on the call's stream and released on it; the pool keeps released
 * memory for later calls (it holds its peak size until mpdd_destroy).  Calls
 * on one handle may be made from several host threads and streams at once.
 */
#ifndef MPDD_H
#define MPDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int64_t mpdd_int;                   /* MPBLAS mplapackint on Linux: 64-bit */
typedef struct { double hi, lo; } mpdd_dd;  /* scalar dd, normalised */
typedef struct mpdd_handle_s *mpdd_handle;

#define MPDD_ERR_HIP (-1)         /* a HIP runtime call or kernel launch failed */
#define MPDD_ERR_ALLOC (-2)       /* device scratch allocation failed */
#define MPDD_ERR_BUDGET (-3)      /* request larger than the server's memory budget */
#define MPDD_ERR_SHUTDOWN (-4)    /* server is shutting down */
#define MPDD_ERR_UNSUPPORTED (-5) /* option value or size outside what is implemented */
#define MPDD_ERR_HANDLE (-6)      /* NULL or destroyed handle */
#define MPDD_ERR_ARG (-7)         /* invalid non-BLAS argument (options, ticket, pointer) */
#define MPDD_ERR_SCRATCH (-8)     /* mpdd_Rgemm_noalloc: needs more than its static scratch */

/* Create a handle bound to the current HIP device.  tuner_cache_path may be
 * NULL (built-in tile choices) or a JSON file written by the autotuner.
 * Returns 0 or MPDD_ERR_*. */
int mpdd_create(mpdd_handle *h, const char *tuner_cache_path);

/* Destroy a handle.  The caller must have synchronised the streams it used. */
int mpdd_destroy(mpdd_handle h);

/* Rgemm: C <- alpha*op(A)*op(B) + beta*C on dd planes (see above).
 * op(A) is m x k, op(B) is k x n, C is m x n.  A is lda x (k or m) for
 * transa N or T, B is ldb x (n or k) for transb N or T. */
int mpdd_Rgemm(mpdd_handle h, const char *transa, const char *transb, mpdd_int m, mpdd_int n,
               mpdd_int k, mpdd_dd alpha, const double *A_hi, const double *A_lo, mpdd_int lda,
               const double *B_hi, const double *B_lo, mpdd_int ldb, mpdd_dd beta,
               double *C_hi, double *C_lo, mpdd_int ldc, void *stream);

/* Rsyrk: C <- alpha*A*A^T + beta*C (trans N, A is n x k) or
 * C <- alpha*A^T*A + beta*C (trans T/C, A is k x n), uplo triangle only. */
int mpdd_Rsyrk(mpdd_handle h, const char *uplo, const char *trans, mpdd_int n, mpdd_int k,
               mpdd_dd alpha, const double *A_hi, const double *A_lo, mpdd_int lda,
               mpdd_dd beta, double *C_hi, double *C_lo, mpdd_int ldc, void *stream);

/* ---- MPBLAS-shaped host entry points ---------------------------------------------
 *
 * The manual's MPBLAS Rgemm / Rsyrk take dd_real arrays in host memory (QD's
 * layout: each entry a {hi, lo} pair of binary64, column-major with a
 * leading dimension; sections "How to use reference MPBLAS" and "CUDA
 * accelerated MPBLAS", where the CUDA dd library replaces the CPU one behind
 * the same prototype).  These entry points take exactly that: A, B, C are
 * HOST pointers to mpdd_dd arrays.  The call copies the operands to the
 * device, runs mpdd_Rgemm / mpdd_Rsyrk, copies C back and returns when C is
 * complete (synchronous).  Same info codes and BLAS semantics as the device
 * calls.  Every array is accessed over its BLAS extent only, ld*(cols-1) + rows
 * entries (a tightly sized array is enough); C is copied both ways over that
 * extent, so padding rows inside it and (Rsyrk) the opposite triangle come
 * back unchanged, and nothing past it is read or written.  Scratch device memory
 * is allocated and freed inside the call.  Copies go through two rings (one
 * per direction) of four 16 MiB pinned host buffers, each with three copy
 * threads, owned by the handle (created by its first host-pointer call,
 * released by mpdd_destroy); the host-pointer calls on one handle are
 * serialised.  Rgemm works on up to 8 column chunks of B and C (at least 512
 * columns each): the copies of one chunk in overlap the product of the
 * previous one on a second stream and the copy of the one before back (a
 * helper thread, a third stream), and with transa = 'N' and k >= 1024 the
 * first chunk is multiplied in k-slices as the matching columns of A arrive
 * (its C accumulated over the slices). */
int mpdd_Rgemm_host(mpdd_handle h, const char *transa, const char *transb, mpdd_int m,
                    mpdd_int n, mpdd_int k, mpdd_dd alpha, const mpdd_dd *A, mpdd_int lda,
                    const mpdd_dd *B, mpdd_int ldb, mpdd_dd beta, mpdd_dd *C, mpdd_int ldc);
int mpdd_Rsyrk_host(mpdd_handle h, const char *uplo, const char *trans, mpdd_int n, mpdd_int k,
                    mpdd_dd alpha, const mpdd_dd *A, mpdd_int lda, mpdd_dd beta, mpdd_dd *C,
                    mpdd_int ldc);

/* ---- explicit algorithm and tile choice ------------------------------------ */

#define MPDD_PLAIN 0          /* lean dd multiply-accumulate (10 binary64 ops per
                                 term; tile entry 4 runs 2 of them, the cross
                                 terms, on the FP64 matrix cores) */
#define MPDD_OZAKI_I8 1       /* split form, INT8 slices on the INT8 matrix cores */
#define MPDD_OZAKI_F64 2      /* split form, FP64 slices on the FP64 matrix cores */
#define MPDD_COMPLEX_3M 4     /* Cgemm only: three real products (see mpdd_Cgemm_ex) */
#define MPDD_PLAIN_ACCURATE 3 /* accurate dd add + mul per term (same steps as the
                                 reference evaluation; 29 binary64 ops) */
#define MPDD_OZAKI_CRT 5      /* split form, residues modulo nslices pairwise coprime
                                 moduli <= 256 on the INT8 matrix cores, one product
                                 per modulus, Chinese-remainder reconstruction (see
                                 mpdd_ozaki_crt_exponent) */

typedef struct {
  int algo;     /* MPDD_PLAIN, MPDD_OZAKI_I8, MPDD_OZAKI_F64, MPDD_OZAKI_CRT,
                   MPDD_PLAIN_ACCURATE */
  int nslices;  /* split form: slices per operand (MPDD_OZAKI_CRT: moduli, 1..32),
                   0 = default for the input */
  int tile_id;  /* plain forms: index into the tile table, -1 = tuned choice;
                   INT8 split form: product workgroup tile, 0 = 256x256,
                   1 = 256x128, 2 = 128x128, 3 = 256x256 with 8 waves,
                   4 = 256x256 with 16 waves, 5 = 256x256 with 8 waves
                   and digits loaded straight into LDS, 6 = as 5 with
                   the next step's fragments read during the MFMAs,
                   7 = as 6 with 4 waves (128x128 each), 8 = as 6 with
                   32x32x32 matrix instructions, -1 = default (6);
                   all give the same bits; MPDD_OZAKI_CRT: 5, 6 or 8
                   (-1 = 6), others MPDD_ERR_UNSUPPORTED; ignored by
                   the FP64 split form */
  int splitk;   /* plain forms: k-split factor, 0 = automatic, 1 = none */
} mpdd_opts;

/* As mpdd_Rgemm with explicit options (opts may be NULL = defaults).
 * Returns MPDD_ERR_ARG for an unknown algo, MPDD_ERR_UNSUPPORTED for an
 * out-of-range tile_id / splitk / nslices. */
int mpdd_Rgemm_ex(mpdd_handle h, const mpdd_opts *opts, const char *transa, const char *transb,
                  mpdd_int m, mpdd_int n, mpdd_int k, mpdd_dd alpha, const double *A_hi,
                  const double *A_lo, mpdd_int lda, const double *B_hi, const double *B_lo,
                  mpdd_int ldb, mpdd_dd beta, double *C_hi, double *C_lo, mpdd_int ldc,
                  void *stream);

/* ---- no-allocation Rgemm ----------------------------------------------------------
 *
 * For callers that cannot allocate device memory during a call: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same product as mpdd_Rgemm_ex with a plain form (opts->algo MPDD_PLAIN
 * or MPDD_PLAIN_ACCURATE; NULL = defaults), same arguments, info codes, BLAS
 * semantics and tile / k-split choice, but the call allocates nothing: its
 * k-split partial sums (16*S*m*n bytes for a split into S k-ranges) go to a
 * static device array of MPDD_STATIC_SCRATCH_BYTES that the library holds on
 * every device it runs on until the process ends (its address is looked up
 * by mpdd_create).  An automatic split whose partials would not fit is halved
 * until they do (S = 1 needs no scratch), so the result is that of
 * mpdd_Rgemm_ex with opts->splitk set to the split used; an explicit
 * opts->splitk whose partials do not fit returns MPDD_ERR_SCRATCH with nothing
 * enqueued.  The split forms return MPDD_ERR_UNSUPPORTED (their slices need
 * far more memory).  Every call on one device shares that device's array,
 * which keeps the last call's contents (nothing in it needs to start at
 * zero): calls whose work may overlap on one device -- on different streams
 * or host threads without an ordering between them -- race on it and must be
 * serialised by the caller (one stream, or events). */
#define MPDD_STATIC_SCRATCH_BYTES ((size_t)64 << 20)   /* 64 MiB per device */

int mpdd_Rgemm_noalloc(mpdd_handle h, const mpdd_opts *opts, const char *transa,
                       const char *transb, mpdd_int m, mpdd_int n, mpdd_int k, mpdd_dd alpha,
                       const double *A_hi, const double *A_lo, mpdd_int lda,
                       const double *B_hi, const double *B_lo, mpdd_int ldb, mpdd_dd beta,
                       double *C_hi, double *C_lo, mpdd_int ldc, void *stream);

/* As mpdd_Rsyrk with explicit options.  The split forms (MPDD_OZAKI_I8 /
 * MPDD_OZAKI_F64 / MPDD_OZAKI_CRT, see the split-form building blocks below)
 * slice op(A) once (the modular form: its residues) and use its slices and
 * row exponents for op(B) = op(A)^T as well, compute
 * only the slice products of the tiles that meet the uplo triangle, and
 * read and write only that triangle of C; their result is that of the
 * split-form mpdd_Rgemm_ex of op(A) and op(A)^T, on the triangle.  INT8
 * product tiling tile_id 1 (256 x 128 tiles) returns MPDD_ERR_UNSUPPORTED
 * here (a triangle is walked in square tiles). */
int mpdd_Rsyrk_ex(mpdd_handle h, const mpdd_opts *opts, const char *uplo, const char *trans,
                  mpdd_int n, mpdd_int k, mpdd_dd alpha, const double *A_hi,
                  const double *A_lo, mpdd_int lda, mpdd_dd beta, double *C_hi,
                  double *C_lo, mpdd_int ldc, void *stream);

/* The host-pointer calls with explicit options: mpdd_Rgemm_host /
 * mpdd_Rsyrk_host (same arguments, info codes, copies and pipelining) whose
 * device products are mpdd_Rgemm_ex / mpdd_Rsyrk_ex with opts (NULL =
 * defaults); an option the device call rejects returns its code with C
 * unchanged.  With a split form Rgemm does not multiply its first column
 * chunk in k-slices (the split scales each row of op(A) over all of k and
 * sizes its slices or moduli for k), so every chunk gets the same exponents,
 * slices or moduli as one device call on the whole matrix and C is bit for
 * bit that call's result; the copies then overlap the products of the later
 * chunks only.  Meant for the split forms, whose device time at large sizes
 * falls below the time of the copies. */
int mpdd_Rgemm_host_ex(mpdd_handle h, const mpdd_opts *opts, const char *transa,
                       const char *transb, mpdd_int m, mpdd_int n, mpdd_int k, mpdd_dd alpha,
                       const mpdd_dd *A, mpdd_int lda, const mpdd_dd *B, mpdd_int ldb,
                       mpdd_dd beta, mpdd_dd *C, mpdd_int ldc);
int mpdd_Rsyrk_host_ex(mpdd_handle h, const mpdd_opts *opts, const char *uplo,
                       const char *trans, mpdd_int n, mpdd_int k, mpdd_dd alpha,
                       const mpdd_dd *A, mpdd_int lda, mpdd_dd beta, mpdd_dd *C, mpdd_int ldc);

/* ---- complex dd: Cgemm ------------------------------------------------------------
 *
 * Cgemm: C <- alpha*op(A)*op(B) + beta*C on complex dd values (manual,
 * section "How to use reference MPBLAS", the Cgemm part: ZGEMM's argument
 * list with complex multiple-precision scalars and arrays).  op(X) = X for
 * 'N', X^T for 'T', the conjugate transpose X^H for 'C' (first character,
 * case-insensitive).  Every complex matrix is four DEVICE planes of binary64
 * -- re.hi, re.lo, im.hi, im.lo -- each column-major with the matrix's
 * leading dimension; sizes and leading dimensions as for mpdd_Rgemm.  Info
 * codes, NULL rules (A and B may be NULL when alpha = 0 or k = 0), beta = 0
 * (C not read) and quick returns (m = 0, n = 0, or (alpha = 0 or k = 0) and
 * beta = 1) are ZGEMM's.  The product op(A) op(B) is formed by four real
 * products on the plain dd kernels into a device scratch of 32*m*n bytes
 * (stream-ordered allocation, released before return), then
 * alpha*P + beta*C is formed in complex dd arithmetic.  Stream-ordered and
 * asynchronous like mpdd_Rgemm; the caller owns every buffer. */
typedef struct { mpdd_dd re, im; } mpdd_ddc;   /* complex dd scalar */

int mpdd_Cgemm(mpdd_handle h, const char *transa, const char *transb, mpdd_int m, mpdd_int n,
               mpdd_int k, mpdd_ddc alpha, const double *A_re_hi, const double *A_re_lo,
               const double *A_im_hi, const double *A_im_lo, mpdd_int lda,
               const double *B_re_hi, const double *B_re_lo, const double *B_im_hi,
               const double *B_im_lo, mpdd_int ldb, mpdd_ddc beta, double *C_re_hi,
               double *C_re_lo, double *C_im_hi, double *C_im_lo, mpdd_int ldc, void *stream);

/* As mpdd_Cgemm with options (NULL = defaults): opts->algo MPDD_PLAIN (the
 * four real products above) or MPDD_COMPLEX_3M (three real products:
 * R1 = Ar Br, R2 = Ai Bi, R3 = (Ar + Ai)(Br + Bi) with the conjugation signs,
 * Re P = R1 - R2, Im P = R3 - R1 - R2; a quarter less arithmetic, with the
 * error of Im P relative to |Ar + Ai| |Br + Bi|; extra scratch
 * 16 (m k + k n) bytes); tile_id / splitk choose the real products' tiling as
 * in mpdd_Rgemm_ex.  MPDD_OZAKI_CRT: the modular split form on complex
 * operands -- one exponent per row of op(A) (column of op(B)) over both
 * parts, grid integers per part (a conjugated operand negates the imaginary
 * ones), three residue products per modulus, T1 = Ar'Br', T2 = Ai'Bi',
 * T3 = (Ar' + Ai')(Br' + Bi'), and Re = T1 - T2, Im = T3 - T1 - T2 rebuilt
 * exactly (P from 8 k 2^(2P) <= M; nslices 0 = the fewest moduli whose P
 * reaches 104), then the same complex epilogue; tile_id 5, 6 or 8.
 * MPDD_OZAKI_I8 / MPDD_OZAKI_F64: the four
 * real products of MPDD_PLAIN, each a split-form product (opts->nslices, tile_id as in
 * mpdd_Rgemm_ex), then the same complex epilogue.  MPDD_ERR_ARG for another
 * algo. */
int mpdd_Cgemm_ex(mpdd_handle h, const mpdd_opts *opts, const char *transa, const char *transb,
                  mpdd_int m, mpdd_int n, mpdd_int k, mpdd_ddc alpha, const double *A_re_hi,
                  const double *A_re_lo, const double *A_im_hi, const double *A_im_lo,
                  mpdd_int lda, const double *B_re_hi, const double *B_re_lo,
                  const double *B_im_hi, const double *B_im_lo, mpdd_int ldb, mpdd_ddc beta,
                  double *C_re_hi, double *C_re_lo, double *C_im_hi, double *C_im_lo,
                  mpdd_int ldc, void *stream);

/* ---- quad-double: Qgemm --------------------------------------------------------------
 *
 * Rgemm on quad-double values (manual, section "Supported Floating point
 * formats": qd_real, four binary64 numbers x0 + x1 + x2 + x3, about 64 digits,
 * epsilon 2^-209 in Table "rlamch_qd"; MPBLAS provides the same Rgemm for
 * qd_real as for dd_real, section "How to use reference MPBLAS").
 * C <- alpha*op(A)*op(B) + beta*C with DGEMM's arguments, info codes, NULL
 * rules and quick returns.  Every matrix is four DEVICE planes (x0, x1, x2,
 * x3), each column-major with the matrix's leading dimension; alpha and beta
 * are qd scalars by value.  Inputs are assumed normalised (|x_{t+1}| <= half
 * an ulp of x_t); outputs are.  Stream-ordered and asynchronous, no scratch. */
typedef struct { double x[4]; } mpdd_qd;       /* quad-double scalar */

int mpdd_Qgemm(mpdd_handle h, const char *transa, const char *transb, mpdd_int m, mpdd_int n,
               mpdd_int k, mpdd_qd alpha, const double *A0, const double *A1, const double *A2,
               const double *A3, mpdd_int lda, const double *B0, const double *B1,
               const double *B2, const double *B3, mpdd_int ldb, mpdd_qd beta, double *C0,
               double *C1, double *C2, double *C3, mpdd_int ldc, void *stream);

/* As mpdd_Qgemm with options (opts may be NULL = MPDD_PLAIN, the kernel
 * above).  opts->algo MPDD_OZAKI_I8: the split form (see the split-form
 * building blocks below) for quad-double operands -- every row of op(A) and
 * column of op(B) is scaled by the exponent of its largest |x0| and cut into
 * opts->nslices INT8 digit slices (0 = 32; at most 48; digit widths as
 * mpdd_ozaki_digit_widths gives them for k), the same exact slice products
 * per anti-diagonal as the dd split form, then the anti-diagonal sums are
 * added in qd from the smallest weight up, scaled back and C = alpha P +
 * beta C is formed in qd.  Device scratch of about
 * nslices ((m + n) k + 4 m n) bytes (padded), stream ordered.  MPDD_ERR_ARG
 * for another algo; MPDD_ERR_UNSUPPORTED for a slice count or tile_id out
 * of range or nslices * k >= 2^19.
 * opts->algo MPDD_OZAKI_CRT: the modular form -- each entry becomes the
 * integer X' = sum_p rint(x_p 2^(208 - sigma)) (sigma from the row's largest
 * |x0|), cut at 2^104 into X1 2^104 + X0 by 26-bit chunks; residues of X1,
 * X0 and X1 + X0 modulo opts->nslices moduli (0 = the fewest that recover
 * the sub-products: M >= 2^(215 + ceil(log2 k)), 30 at k = 2048; fewer return
 * MPDD_ERR_UNSUPPORTED), three INT8 residue products per modulus, the exact
 * product A 2^208 + (C - A - B) 2^104 + B rebuilt from A = X1 Y1, B = X0 Y0,
 * C = (X1 + X0)(Y1 + Y0), summed into a qd, scaled back, C = alpha P +
 * beta C in qd; tile_id 5, 6 or 8; k < 2^17. */
int mpdd_Qgemm_ex(mpdd_handle h, const mpdd_opts *opts, const char *transa, const char *transb,
                  mpdd_int m, mpdd_int n, mpdd_int k, mpdd_qd alpha, const double *A0,
                  const double *A1, const double *A2, const double *A3, mpdd_int lda,
                  const double *B0, const double *B1, const double *B2, const double *B3,
                  mpdd_int ldb, mpdd_qd beta, double *C0, double *C1, double *C2, double *C3,
                  mpdd_int ldc, void *stream);

/* ---- Cholesky factorisation: Rpotrf -------------------------------------------------
 *
 * Rpotrf: the dd Cholesky factorisation of a symmetric positive definite
 * matrix (MPLAPACK's Rpotrf, LAPACK DPOTRF's argument list: uplo, n, A, lda,
 * info; the manual lists it among the MPLAPACK routines and times it on the
 * CPU; the interior-point (SDP) solvers it cites factor their Schur
 * complement matrices this way).  uplo 'L': A = L L^T, L written over the
 * lower triangle; 'U': A = U^T U over the upper triangle.  A is two DEVICE
 * planes (hi, lo), column-major, n x n with leading dimension lda; only the
 * uplo triangle is read or written.
 *
 * *info (HOST pointer, required) receives LAPACK's info: 0; -1 (uplo),
 * -2 (n < 0), -4 (lda < max(1, n)) with nothing enqueued; or k > 0 when the
 * leading minor of order k is not positive definite (pivot <= 0 or NaN): the
 * columns before k's block hold the factor, A(k,k) holds the pivot, later
 * columns are unspecified.  The return value is 0 or MPDD_ERR_* (library /
 * runtime errors only).
 *
 * Blocked: per diagonal block of order nb, Rgemm calls update a copy of the
 * block column (the bulk of them on two internal streams that overlap the
 * work on `stream`), a one-workgroup kernel factors the diagonal block and
 * inverts its factor, and the rest of the block column is multiplied by the
 * inverted block.  The call reads the failure word back to the host every 16
 * blocks and at the end, so it is synchronous: it returns when A is factored
 * (or a failing pivot has been found).  Device scratch of 16*nb*(nb + 3n) +
 * 256 bytes, plus the k-split partial sums of the update products, is
 * allocated and freed inside the call (stream ordered). */
int mpdd_Rpotrf(mpdd_handle h, const char *uplo, mpdd_int n, double *A_hi, double *A_lo,
                mpdd_int lda, mpdd_int *info, void *stream);

/* As mpdd_Rpotrf with the block order nb (1..64; 0 = default 64);
 * MPDD_ERR_UNSUPPORTED outside that range. */
int mpdd_Rpotrf_nb(mpdd_handle h, const char *uplo, mpdd_int n, double *A_hi, double *A_lo,
                   mpdd_int lda, mpdd_int nb, mpdd_int *info, void *stream);

/* As mpdd_Rpotrf_nb with options (opts may be NULL = MPDD_PLAIN, the form
 * above).  opts->algo MPDD_OZAKI_I8 / MPDD_OZAKI_F64 / MPDD_OZAKI_CRT:
 * right-looking over
 * panels of 1024 columns (rounded down to whole blocks) -- each panel is factored
 * as above inside the trailing matrix, then the rest of the trailing matrix
 * takes the panel's update in one split-form mpdd_Rsyrk_ex with
 * opts->nslices slices or moduli (lower: A22 -= L21 L21^T; upper:
 * A22 -= U12^T U12);
 * the panels are enqueued without host round trips and the failure word is
 * read once, at the end.  Same arguments, info and synchronisation as
 * mpdd_Rpotrf; MPDD_ERR_ARG for any other algo; errors of a trailing update
 * are returned as they are. */
int mpdd_Rpotrf_ex(mpdd_handle h, const mpdd_opts *opts, const char *uplo, mpdd_int n,
                   double *A_hi, double *A_lo, mpdd_int lda, mpdd_int nb, mpdd_int *info,
                   void *stream);

/* ---- split-form building blocks ------------------------------------------------ *
 *
 * The split form (algo MPDD_OZAKI_I8 / MPDD_OZAKI_F64) cuts every row of op(A)
 * and every column of op(B) into `nslices` digit slices: with sigma the
 * frexp exponent of the row's largest |hi| (so |x| < 2^sigma), y = x 2^-sigma
 * and, for t = 1..nslices, z = y 2^w_t, q_t = rint(z.hi), y = TwoSum(z.hi - q_t,
 * z.lo).  INT8: w_1 = 6 and w_t = 8 while nslices*k < 2^17 -- a later digit
 * above 127 (it rounds to 128, or a carry lifts a 127) loses 256 and the digit
 * before it gains one, from the last digit up, so later digits lie in
 * [-128, 127] -- else w_t = 7 (|q| <= 64).  FP64: w_1 = w - 1, w_t = w, with
 * w = floor((55 - ceil(log2(nslices*k))) / 2) so that sums of nslices*k digit
 * products are exact in binary64.  Slice products are accumulated exactly per
 * anti-diagonal on the matrix cores and recombined in dd (published basis:
 * Ozaki, Ogita, Oishi, Rump 2012; Ootomo, Ozaki, Yokota 2024 -- the manual
 * itself has no split method). */

/* Digit widths (first, later) of a split form for k and nslices.
 * Returns 0, or MPDD_ERR_UNSUPPORTED when no exact width exists (INT8 needs
 * nslices*k < 2^19, so that every anti-diagonal sum, at most
 * nslices*k*2^(2w-2) in magnitude, stays below 2^31: w = 8 below 2^17,
 * w = 7 from there). */
int mpdd_ozaki_digit_widths(int algo, mpdd_int k, int nslices, int *wfirst, int *w);

/* The modular split form (algo MPDD_OZAKI_CRT; published basis: the integer
 * modular emulation of Ozaki, Uchino and Imamura, "Ozaki scheme II", 2025).
 * With sigma as above and P = mpdd_ozaki_crt_exponent(k, nslices), each
 * element becomes the integer x' = t1 + t2, z = x 2^(P - sigma) (binary64
 * parts zh + zl), t1 = rint(zh), t2 = rint((zh - t1) + zl), so |x' - z| <=
 * 1/2 + 2^-52 and |x'| <= 2^P.  The moduli are 256, 255, 253, 251, 247, ...:
 * from 256 down, each integer coprime to all moduli before it; the first
 * nslices are used, M their product.  x' is reduced to balanced residues
 * (odd m: [-(m-1)/2, (m-1)/2]; 256: [-128, 127]), one exact INT8 product per
 * modulus gives the integer product modulo that modulus, and the exact
 * integer product (|.| <= k 2^(2P) <= M/4) is rebuilt by Chinese
 * remaindering and rounded to dd, then scaled by 2^(sigma_i + tau_j - 2P) and
 * C = alpha P + beta C.  Error against the exact product of the dd inputs:
 * at most sum_l (|dA_il| |B_lj| + |A_il| |dB_lj| + |dA_il| |dB_lj|) with
 * |dA_il| <= (1/2 + 2^-52) 2^(sigma_i - P), plus dd rounding.  k must be
 * below 2^17 (k 128^2 < 2^31).  nslices 0 = the fewest moduli whose P
 * reaches 104 (30 at k = 8192). */

/* P of the modular split form: the largest P <= 104 with 4 k 2^(2P) <= M for
 * the first nmoduli moduli.  Returns 0, MPDD_ERR_ARG for k < 0, a NULL p or
 * nmoduli outside 1..32, MPDD_ERR_UNSUPPORTED when k >= 2^17 or no P >= 1
 * fits. */
int mpdd_ozaki_crt_exponent(mpdd_int k, int nmoduli, int *p);

/* Scale exponents and digit slices of a "row operand" R (rows x k): element
 * (r, l) of R is X[r + l*ld] for trans "N" and X[l + r*ld] for trans "T"
 * (rows of op(A) are R with trans = transa; columns of op(B) are R with the
 * flag opposite to transb).  Device outputs: exps[rows] (int32) and
 * `nslices` planes of rows_p x ldq digits, plane t (0-based) at
 * slices + t*rows_p*ldq, digit (r, l) at [r*ldq + l]; int8 for
 * MPDD_OZAKI_I8, double for MPDD_OZAKI_F64; for MPDD_OZAKI_CRT the planes are
 * the int8 balanced residues of x' modulo the first `nslices` moduli (1..32),
 * plane t for modulus t.  ldq must be a multiple of 64 and
 * >= k, rows_p a multiple of 64 and >= rows; padding digits are written as 0.
 * Returns 0, a BLAS-style position (3 rows, 4 k, 8 ld, 9 nslices, 12 ldq,
 * 13 rows_p) for an invalid argument, or MPDD_ERR_*. */
int mpdd_ozaki_split(mpdd_handle h, int algo, const char *trans, mpdd_int rows, mpdd_int k,
                     const double *X_hi, const double *X_lo, mpdd_int ld, int nslices,
                     int *exps, void *slices, mpdd_int ldq, mpdd_int rows_p, void *stream);

/* ---- request server (continuous batching) ----------------------------------------
 *
 * A server owns a scheduler thread and four slot streams.  Submitted requests
 * are validated (same info codes as the plain calls), admitted in FIFO order
 * while the memory budget allows -- a request counts 16 bytes per dd entry
 * of A, B and C (ld x columns) from admission to completion, and requests
 * larger than the whole budget fail with MPDD_ERR_BUDGET -- and launched as
 * groups: all admitted requests go into one persistent grouped kernel launch
 * (a captured hipGraph) on a free slot, so groups overlap on the device and
 * new requests start as soon as a slot and budget free up.  Each result is
 * bit-identical to a standalone mpdd_Rgemm_ex / mpdd_Rsyrk_ex with the same
 * tile (the server uses the handle's tuned tile, restricted to tile-table
 * entries 2 and 4: 32 x 32 and 64 x 64 x 16).  Operands stay where the
 * caller put them (device memory) and must stay valid until the request
 * completes.  A group of one request is launched as a plain tile kernel;
 * when the server is idle (nothing queued or admitted, a slot free) and the
 * submitting thread has the server's device current, submit launches the
 * request itself instead of handing it to the scheduler thread.
 * The scheduler thread polls (yielding its core) while work is in flight and
 * for 50 ms after its last activity, then sleeps until the next submission.
 *
 * Intended callers: any host thread; submit and wait may run concurrently. */

#define MPDD_OP_GEMM 0
#define MPDD_OP_SYRK 1

typedef struct mpdd_server_s *mpdd_server;

typedef struct {
  int op;                  /* MPDD_OP_GEMM or MPDD_OP_SYRK */
  char flag1, flag2;       /* Rgemm: transa, transb; Rsyrk: uplo, trans */
  char pad_[2];
  mpdd_int m, n, k;        /* Rsyrk: n, k (m ignored) */
  mpdd_dd alpha, beta;
  const double *A_hi, *A_lo;
  mpdd_int lda;
  const double *B_hi, *B_lo;   /* Rgemm only */
  mpdd_int ldb;
  double *C_hi, *C_lo;
  mpdd_int ldc;
  double arrival;          /* arrival time on mpdd_clock(); < 0 = time of submit */
  int inject;              /* 0; other values are test hooks (mpdd_testing.h) */
  int pad2_;
} mpdd_request;

typedef struct {
  double arrival, submit, admit, start, end;   /* mpdd_clock() seconds */
  int group;                                   /* group the request ran in (0: none) */
  int info;                                    /* the request's info code */
  int tile;                                    /* tile-table id it ran with (-1: none) */
  int pad_;
} mpdd_timing;

typedef struct {
  int64_t submitted, completed, failed, groups;
  int64_t queued_requests, inflight_requests;
  uint64_t inflight_bytes;
} mpdd_server_stats;

/* Monotonic clock (seconds) used for request timings. */
double mpdd_clock(void);

/* Create a server on handle h (its device and tuned tiles) with a memory
 * budget and at most max_inflight admitted requests.  flags: 0 (other values
 * are test hooks, mpdd_testing.h).  Returns 0 or MPDD_ERR_*. */
int mpdd_server_create(mpdd_server *s, mpdd_handle h, size_t hbm_budget_bytes, int max_inflight,
                       int flags);

/* Enqueue a request (non-blocking).  *ticket identifies it for wait/poll.
 * Returns 0 (the request's own outcome is reported by wait), MPDD_ERR_ARG,
 * or MPDD_ERR_SHUTDOWN. */
int mpdd_server_submit(mpdd_server s, const mpdd_request *r, uint64_t *ticket);

/* Block until the request completes; report its info code and timings and
 * forget the ticket.  Returns 0 or MPDD_ERR_ARG (unknown ticket). */
int mpdd_server_wait(mpdd_server s, uint64_t ticket, int *info, mpdd_timing *t);

/* *done = 1 if the request has completed (ticket stays valid). */
int mpdd_server_poll(mpdd_server s, uint64_t ticket, int *done);

int mpdd_server_get_stats(mpdd_server s, mpdd_server_stats *st);

/* Drain every queued and in-flight request, then free the server. */
int mpdd_server_destroy(mpdd_server s);

/* Number of entries in the plain-kernel tile table, and a description of
 * entry id: tile rows, tile columns, k-depth of one staged tile, threads per
 * workgroup.  Returns 0 or MPDD_ERR_ARG. */
int mpdd_tile_count(void);
int mpdd_tile_info(int id, int *bm, int *bn, int *bk, int *threads);

/* Library version string (static storage). */
const char *mpdd_version(void);

/* sizeof of an ABI struct by name ("mpdd_dd", "mpdd_opts", "mpdd_request",
 * "mpdd_timing", "mpdd_server_stats"), 0 if unknown: lets bindings check
 * their layouts. */
size_t mpdd_struct_size(const char *name);

#ifdef __cplusplus
}
#endif

#endif /* MPDD_H */

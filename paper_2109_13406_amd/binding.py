"""ctypes binding of libmpdd (include/mpdd.h): argument marshalling only.

Every function named mpdd_* here calls the C entry point of the same name;
all arithmetic runs in the library's HIP kernels.  There is no fallback: if
libmpdd.so is missing or fails to load, load() raises.

Matrices are passed as (hi, lo) pairs of device pointers, or of torch float64
CUDA tensors holding the column-major storage (flat, element (i, j) at
[i + j*ld]); torch provides device memory and streams only.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmpdd.so")

MPDD_PLAIN = 0
MPDD_OZAKI_I8 = 1
MPDD_OZAKI_F64 = 2
MPDD_PLAIN_ACCURATE = 3
MPDD_COMPLEX_3M = 4
MPDD_OZAKI_CRT = 5

MPDD_ERR_HIP = -1
MPDD_ERR_ALLOC = -2
MPDD_ERR_BUDGET = -3
MPDD_ERR_SHUTDOWN = -4
MPDD_ERR_UNSUPPORTED = -5
MPDD_ERR_HANDLE = -6
MPDD_ERR_ARG = -7
MPDD_ERR_SCRATCH = -8
MPDD_STATIC_SCRATCH_BYTES = 64 << 20   # static scratch of mpdd_Rgemm_noalloc, per device


class mpdd_dd(ctypes.Structure):
    _fields_ = [("hi", ctypes.c_double), ("lo", ctypes.c_double)]


class mpdd_ddc(ctypes.Structure):
    _fields_ = [("re", mpdd_dd), ("im", mpdd_dd)]


class mpdd_qd(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double * 4)]


class mpdd_opts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int), ("nslices", ctypes.c_int), ("tile_id", ctypes.c_int),
                ("splitk", ctypes.c_int)]


class mpdd_request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("flag1", ctypes.c_char), ("flag2", ctypes.c_char),
                ("pad_", ctypes.c_char * 2), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("k", ctypes.c_int64), ("alpha", mpdd_dd), ("beta", mpdd_dd),
                ("A_hi", ctypes.c_void_p), ("A_lo", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B_hi", ctypes.c_void_p), ("B_lo", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C_hi", ctypes.c_void_p), ("C_lo", ctypes.c_void_p), ("ldc", ctypes.c_int64),
                ("arrival", ctypes.c_double), ("inject", ctypes.c_int), ("pad2_", ctypes.c_int)]


class mpdd_timing(ctypes.Structure):
    _fields_ = [("arrival", ctypes.c_double), ("submit", ctypes.c_double),
                ("admit", ctypes.c_double), ("start", ctypes.c_double), ("end", ctypes.c_double),
                ("group", ctypes.c_int), ("info", ctypes.c_int), ("tile", ctypes.c_int),
                ("pad_", ctypes.c_int)]


class mpdd_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("groups", ctypes.c_int64),
                ("queued_requests", ctypes.c_int64), ("inflight_requests", ctypes.c_int64),
                ("inflight_bytes", ctypes.c_uint64)]


MPDD_OP_GEMM = 0
MPDD_OP_SYRK = 1
# test hooks of the request server (include/mpdd_testing.h)
MPDD_SERVER_FAKE_DEVICE = 1
MPDD_INJECT_NONE = 0
MPDD_INJECT_DEVICE_ERROR = 1
MPDD_INJECT_ALLOC_FAILURE = 2

_I = ctypes.c_int64
_P = ctypes.c_void_p
_C = ctypes.c_char_p

# name -> (restype, argtypes)
SIGNATURES = {
    "mpdd_version": (ctypes.c_char_p, []),
    "mpdd_create": (ctypes.c_int, [ctypes.POINTER(_P), _C]),
    "mpdd_destroy": (ctypes.c_int, [_P]),
    "mpdd_Rgemm": (ctypes.c_int, [_P, _C, _C, _I, _I, _I, mpdd_dd, _P, _P, _I, _P, _P, _I,
                                  mpdd_dd, _P, _P, _I, _P]),
    "mpdd_Rgemm_ex": (ctypes.c_int, [_P, ctypes.POINTER(mpdd_opts), _C, _C, _I, _I, _I, mpdd_dd,
                                     _P, _P, _I, _P, _P, _I, mpdd_dd, _P, _P, _I, _P]),
    "mpdd_Rgemm_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(mpdd_opts), _C, _C, _I, _I, _I,
                                          mpdd_dd, _P, _P, _I, _P, _P, _I, mpdd_dd, _P, _P, _I,
                                          _P]),
    "mpdd_Rsyrk": (ctypes.c_int, [_P, _C, _C, _I, _I, mpdd_dd, _P, _P, _I, mpdd_dd, _P, _P, _I,
                                  _P]),
    "mpdd_Rsyrk_ex": (ctypes.c_int, [_P, ctypes.POINTER(mpdd_opts), _C, _C, _I, _I, mpdd_dd, _P,
                                     _P, _I, mpdd_dd, _P, _P, _I, _P]),
    "mpdd_Cgemm": (ctypes.c_int, [_P, _C, _C, _I, _I, _I, mpdd_ddc, _P, _P, _P, _P, _I, _P, _P, _P,
                                  _P, _I, mpdd_ddc, _P, _P, _P, _P, _I, _P]),
    "mpdd_Cgemm_ex": (ctypes.c_int, [_P, ctypes.POINTER(mpdd_opts), _C, _C, _I, _I, _I, mpdd_ddc,
                                     _P, _P, _P, _P, _I, _P, _P, _P, _P, _I, mpdd_ddc, _P, _P, _P,
                                     _P, _I, _P]),
    "mpdd_Qgemm": (ctypes.c_int, [_P, _C, _C, _I, _I, _I, mpdd_qd, _P, _P, _P, _P, _I, _P, _P, _P,
                                  _P, _I, mpdd_qd, _P, _P, _P, _P, _I, _P]),
    "mpdd_Qgemm_ex": (ctypes.c_int, [_P, ctypes.POINTER(mpdd_opts), _C, _C, _I, _I, _I, mpdd_qd,
                                     _P, _P, _P, _P, _I, _P, _P, _P, _P, _I, mpdd_qd, _P, _P, _P,
                                     _P, _I, _P]),
    "mpdd_Rpotrf": (ctypes.c_int, [_P, _C, _I, _P, _P, _I, ctypes.POINTER(_I), _P]),
    "mpdd_Rpotrf_nb": (ctypes.c_int, [_P, _C, _I, _P, _P, _I, _I, ctypes.POINTER(_I), _P]),
    "mpdd_Rpotrf_ex": (ctypes.c_int, [_P, ctypes.POINTER(mpdd_opts), _C, _I, _P, _P, _I, _I,
                                      ctypes.POINTER(_I), _P]),
    "mpdd_ozaki_digit_widths": (ctypes.c_int, [ctypes.c_int, _I, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_int)]),
    "mpdd_ozaki_crt_exponent": (ctypes.c_int, [_I, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "mpdd_ozaki_split": (ctypes.c_int, [_P, ctypes.c_int, _C, _I, _I, _P, _P, _I, ctypes.c_int,
                                        _P, _P, _I, _I, _P]),
    "mpdd_Rgemm_host": (ctypes.c_int, [_P, _C, _C, _I, _I, _I, mpdd_dd, _P, _I, _P, _I, mpdd_dd,
                                       _P, _I]),
    "mpdd_Rsyrk_host": (ctypes.c_int, [_P, _C, _C, _I, _I, mpdd_dd, _P, _I, mpdd_dd, _P, _I]),
    "mpdd_Rgemm_host_ex": (ctypes.c_int, [_P, ctypes.POINTER(mpdd_opts), _C, _C, _I, _I, _I,
                                          mpdd_dd, _P, _I, _P, _I, mpdd_dd, _P, _I]),
    "mpdd_Rsyrk_host_ex": (ctypes.c_int, [_P, ctypes.POINTER(mpdd_opts), _C, _C, _I, _I,
                                          mpdd_dd, _P, _I, mpdd_dd, _P, _I]),
    "mpdd_struct_size": (ctypes.c_size_t, [_C]),
    "mpdd_clock": (ctypes.c_double, []),
    "mpdd_server_create": (ctypes.c_int, [ctypes.POINTER(_P), _P, ctypes.c_size_t, ctypes.c_int,
                                          ctypes.c_int]),
    "mpdd_server_set_fake_rate": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double]),
    "mpdd_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(mpdd_request),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "mpdd_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(mpdd_timing)]),
    "mpdd_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]),
    "mpdd_server_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(mpdd_server_stats)]),
    "mpdd_server_destroy": (ctypes.c_int, [_P]),
    "mpdd_tile_count": (ctypes.c_int, []),
    "mpdd_tile_info": (ctypes.c_int, [ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 4),
}

_LIB = None


def load():
    """Load libmpdd.so (raises OSError / RuntimeError when it is missing)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2109_13406_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _LIB = lib
    return _LIB


def _ptr(x):
    """Device pointer of a torch tensor, an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _extent(rows, cols, ld):
    """Elements spanned by a column-major rows x cols matrix with leading
    dimension ld (0 when it is empty)."""
    return 0 if rows <= 0 or cols <= 0 else ld * (cols - 1) + rows


def _first(flag):
    if isinstance(flag, bytes):
        flag = flag.decode(errors="replace")
    return flag[:1].upper() if isinstance(flag, str) else ""


def _dev(x, need, name, dtype=None):
    """Pointer for a device argument that the call will touch over `need`
    elements: a CUDA tensor of the expected dtype (float64 unless given),
    contiguous, with at least `need` elements from its start, is checked
    before the library sees it, since the kernels cannot tell a host pointer
    or a short buffer from a good one.  Raw integer pointers and None pass
    unchecked, and so does an argument the call does not touch (need 0)."""
    if x is None or isinstance(x, int) or need <= 0:
        return _ptr(x)
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor or a device pointer, got {type(x)}")
    want = dtype or torch.float64
    if x.dtype != want:
        raise ValueError(f"{name}: dtype {x.dtype}, expected {want}")
    if not x.is_cuda:
        raise ValueError(f"{name}: tensor on {x.device}, expected a CUDA device")
    if not x.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous (column-major planes with ld)")
    if x.numel() < need:
        raise ValueError(f"{name}: {x.numel()} elements, the call touches {need}")
    return x.data_ptr()


def _planes(xs, need, name):
    return [_dev(x, need, f"{name}[{i}]") for i, x in enumerate(xs)]


def _gemm_extents(transa, transb, m, n, k, lda, ldb, ldc):
    """(A, B, C) element extents of a valid Rgemm-shaped call, or None when an
    argument is invalid (the library then returns its info code)."""
    fa, fb = _first(transa), _first(transb)
    if fa not in ("N", "T", "C") or fb not in ("N", "T", "C") or min(m, n, k) < 0:
        return None
    nra, nca = (m, k) if fa == "N" else (k, m)
    nrb, ncb = (k, n) if fb == "N" else (n, k)
    if lda < max(1, nra) or ldb < max(1, nrb) or ldc < max(1, m):
        return None
    return _extent(nra, nca, lda), _extent(nrb, ncb, ldb), _extent(m, n, ldc)


def _syrk_extents(uplo, trans, n, k, lda, ldc):
    """(A, C) element extents of a valid Rsyrk call, or None."""
    fu, ft = _first(uplo), _first(trans)
    if fu not in ("U", "L") or ft not in ("N", "T", "C") or min(n, k) < 0:
        return None
    nra, nca = (n, k) if ft == "N" else (k, n)
    if lda < max(1, nra) or ldc < max(1, n):
        return None
    return _extent(nra, nca, lda), _extent(n, n, ldc)


def _touches(ext, alpha_zero, beta_one, k, m, n):
    """Extents actually read / written: (A and B, C).  A and B are not read
    when alpha = 0 or k = 0; C is not touched on a quick return."""
    if ext is None or m == 0 or n == 0:
        return 0, 0
    ab = not (alpha_zero or k == 0)
    c_touched = ab or not beta_one
    return ab, c_touched


def _gemm_ptrs(nplanes, transa, transb, m, n, k, alpha_zero, beta_one, A, lda, B, ldb, C, ldc):
    ext = _gemm_extents(transa, transb, m, n, k, lda, ldb, ldc)
    ab, ct = _touches(ext, alpha_zero, beta_one, k, m, n)
    ea, eb, ec = ext if ext else (0, 0, 0)
    assert len(A) == nplanes and len(B) == nplanes and len(C) == nplanes
    return (_planes(A, ea if ab else 0, "A"), _planes(B, eb if ab else 0, "B"),
            _planes(C, ec if ct else 0, "C"))


def _dd(x):
    if isinstance(x, mpdd_dd):
        return x
    if isinstance(x, (int, float)):
        return mpdd_dd(float(x), 0.0)
    return mpdd_dd(float(x[0]), float(x[1]))


def _ddc(x):
    """complex dd scalar: mpdd_ddc, a Python complex / real number (binary64
    parts), or ((re_hi, re_lo), (im_hi, im_lo))."""
    if isinstance(x, mpdd_ddc):
        return x
    if isinstance(x, (int, float, complex)):
        x = complex(x)
        return mpdd_ddc(mpdd_dd(x.real, 0.0), mpdd_dd(x.imag, 0.0))
    return mpdd_ddc(_dd(x[0]), _dd(x[1]))


def _flag(s):
    return s.encode() if isinstance(s, str) else s


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _opts(algo=MPDD_PLAIN, nslices=0, tile_id=-1, splitk=0):
    return mpdd_opts(algo, nslices, tile_id, splitk)


# ---- the C entry points, same names -------------------------------------------

def mpdd_version():
    return load().mpdd_version().decode()


def mpdd_create(tuner_cache_path=None):
    h = _P()
    info = load().mpdd_create(ctypes.byref(h),
                              tuner_cache_path.encode() if tuner_cache_path else None)
    if info != 0:
        raise RuntimeError(f"mpdd_create failed: {info}")
    return h


def mpdd_destroy(h):
    return load().mpdd_destroy(h)


def _dd_zero(x):
    return x.hi == 0.0 and x.lo == 0.0


def _dd_one(x):
    return x.hi == 1.0 and x.lo == 0.0


def mpdd_Rgemm(h, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    """A, B, C: (hi, lo) pairs of tensors or device pointers.  Returns info."""
    return mpdd_Rgemm_ex(h, None, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                         stream, _entry="mpdd_Rgemm")


def mpdd_Rgemm_ex(h, opts, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                  stream=None, _entry="mpdd_Rgemm_ex"):
    a, bt = _dd(alpha), _dd(beta)
    pa, pb, pc = _gemm_ptrs(2, transa, transb, m, n, k, _dd_zero(a), _dd_one(bt), A, lda, B, ldb,
                            C, ldc)
    args = (_flag(transa), _flag(transb), m, n, k, a, pa[0], pa[1], lda, pb[0], pb[1], ldb, bt,
            pc[0], pc[1], ldc, _stream(stream))
    if _entry == "mpdd_Rgemm":
        return load().mpdd_Rgemm(h, *args)
    o = opts if opts is None or isinstance(opts, mpdd_opts) else _opts(**opts)
    return getattr(load(), _entry)(h, ctypes.byref(o) if o is not None else None, *args)


def mpdd_Rgemm_noalloc(h, opts, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                       stream=None):
    """As mpdd_Rgemm_ex; the library allocates nothing (k-split partials in
    its static per-device scratch).  Returns info or MPDD_ERR_*."""
    return mpdd_Rgemm_ex(h, opts, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                         stream, _entry="mpdd_Rgemm_noalloc")


def prepared_Rgemm_ex(h, opts, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                      stream=None):
    """The same call as mpdd_Rgemm_ex with every argument checked and
    marshalled now: returns a callable that issues it (returning info).  For
    callers that issue a prepared call at a later moment (a load generator
    pacing requests) without paying the marshalling then."""
    import functools
    a, bt = _dd(alpha), _dd(beta)
    pa, pb, pc = _gemm_ptrs(2, transa, transb, m, n, k, _dd_zero(a), _dd_one(bt), A, lda, B, ldb,
                            C, ldc)
    o = opts if opts is None or isinstance(opts, mpdd_opts) else _opts(**opts)
    return functools.partial(load().mpdd_Rgemm_ex, h, ctypes.byref(o) if o is not None else None,
                             _flag(transa), _flag(transb), m, n, k, a, pa[0], pa[1], lda, pb[0],
                             pb[1], ldb, bt, pc[0], pc[1], ldc, _stream(stream))


def prepared_Rsyrk_ex(h, opts, uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream=None):
    """As prepared_Rgemm_ex, for mpdd_Rsyrk_ex."""
    import functools
    o = opts if opts is None or isinstance(opts, mpdd_opts) else _opts(**opts)
    return functools.partial(load().mpdd_Rsyrk_ex, h, ctypes.byref(o) if o is not None else None,
                             *_syrk_args(uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream))


def _cgemm_args(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream):
    a, bt = _ddc(alpha), _ddc(beta)
    pa, pb, pc = _gemm_ptrs(4, transa, transb, m, n, k, _dd_zero(a.re) and _dd_zero(a.im),
                            _dd_one(bt.re) and _dd_zero(bt.im), A, lda, B, ldb, C, ldc)
    return (_flag(transa), _flag(transb), m, n, k, a, *pa, lda, *pb, ldb, bt, *pc, ldc,
            _stream(stream))


def mpdd_Cgemm(h, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    """A, B, C: 4-tuples (re.hi, re.lo, im.hi, im.lo) of tensors or device
    pointers.  Returns info."""
    return load().mpdd_Cgemm(h, *_cgemm_args(transa, transb, m, n, k, alpha, A, lda, B, ldb,
                                             beta, C, ldc, stream))


def mpdd_Cgemm_ex(h, opts, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                  stream=None):
    o = opts if opts is None or isinstance(opts, mpdd_opts) else _opts(**opts)
    return load().mpdd_Cgemm_ex(h, ctypes.byref(o) if o is not None else None,
                                *_cgemm_args(transa, transb, m, n, k, alpha, A, lda, B, ldb,
                                             beta, C, ldc, stream))


def _qd(x):
    if isinstance(x, mpdd_qd):
        return x
    if isinstance(x, (int, float)):
        x = (float(x), 0.0, 0.0, 0.0)
    return mpdd_qd((ctypes.c_double * 4)(*[float(v) for v in x]))


def mpdd_Qgemm(h, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None,
               opts=None):
    """Quad-double Rgemm.  A, B, C: 4-tuples of planes (x0..x3) as tensors or
    device pointers; alpha, beta: 4-tuples of floats.  With opts (an
    mpdd_opts or a dict of its fields) the call goes to mpdd_Qgemm_ex.
    Returns info."""
    a, bt = _qd(alpha), _qd(beta)
    pa, pb, pc = _gemm_ptrs(4, transa, transb, m, n, k, all(v == 0.0 for v in a.x),
                            list(bt.x) == [1.0, 0.0, 0.0, 0.0], A, lda, B, ldb, C, ldc)
    if opts is None:
        return load().mpdd_Qgemm(h, _flag(transa), _flag(transb), m, n, k, a, *pa, lda, *pb, ldb,
                                 bt, *pc, ldc, _stream(stream))
    o = opts if isinstance(opts, mpdd_opts) else _opts(**opts)
    return load().mpdd_Qgemm_ex(h, ctypes.byref(o), _flag(transa), _flag(transb), m, n, k, a,
                                *pa, lda, *pb, ldb, bt, *pc, ldc, _stream(stream))


def mpdd_Rpotrf(h, uplo, n, A, lda, nb=0, stream=None, opts=None):
    """A: (hi, lo) pair of tensors or device pointers.  Returns (rc, info):
    rc = 0 or MPDD_ERR_*, info = LAPACK's info.  With opts (an mpdd_opts or
    a dict of its fields) the call goes to mpdd_Rpotrf_ex."""
    info = _I(0)
    ok = _first(uplo) in ("U", "L") and n >= 0 and lda >= max(1, n)
    pa = _planes(A, _extent(n, n, lda) if ok else 0, "A")
    if opts is None:
        rc = load().mpdd_Rpotrf_nb(h, _flag(uplo), n, pa[0], pa[1], lda, nb, ctypes.byref(info),
                                   _stream(stream))
    else:
        o = opts if isinstance(opts, mpdd_opts) else _opts(**opts)
        rc = load().mpdd_Rpotrf_ex(h, ctypes.byref(o), _flag(uplo), n, pa[0], pa[1], lda, nb,
                                   ctypes.byref(info), _stream(stream))
    return rc, info.value


def _syrk_args(uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream):
    a, bt = _dd(alpha), _dd(beta)
    ext = _syrk_extents(uplo, trans, n, k, lda, ldc)
    ab, ct = _touches(ext, _dd_zero(a), _dd_one(bt), k, n, n)
    ea, ec = ext if ext else (0, 0)
    pa, pc = _planes(A, ea if ab else 0, "A"), _planes(C, ec if ct else 0, "C")
    return (_flag(uplo), _flag(trans), n, k, a, pa[0], pa[1], lda, bt, pc[0], pc[1], ldc,
            _stream(stream))


def mpdd_Rsyrk(h, uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream=None):
    return load().mpdd_Rsyrk(h, *_syrk_args(uplo, trans, n, k, alpha, A, lda, beta, C, ldc,
                                            stream))


def mpdd_Rsyrk_ex(h, opts, uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream=None):
    o = opts if opts is None or isinstance(opts, mpdd_opts) else _opts(**opts)
    return load().mpdd_Rsyrk_ex(h, ctypes.byref(o) if o is not None else None,
                                *_syrk_args(uplo, trans, n, k, alpha, A, lda, beta, C, ldc,
                                            stream))


def _host_pairs(x, need=0, name="array"):
    """Pointer to an interleaved {hi, lo} host array: a C-contiguous numpy
    float64 array of shape (..., 2) / length 2*count holding at least `need`
    pairs, or None."""
    if x is None:
        return None
    import numpy as np
    if not isinstance(x, np.ndarray) or x.dtype != np.float64 or not x.flags.c_contiguous:
        raise ValueError(f"{name}: expected a C-contiguous numpy float64 array")
    if x.size < 2 * need:
        raise ValueError(f"{name}: {x.size // 2} dd values, the call touches {need}")
    return x.ctypes.data


def _opts_ref(opts):
    o = opts if opts is None or isinstance(opts, mpdd_opts) else _opts(**opts)
    return ctypes.byref(o) if o is not None else None


def mpdd_Rgemm_host(h, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    """MPBLAS-shaped Rgemm on host dd_real arrays (numpy float64, {hi, lo}
    interleaved).  Synchronous; returns info."""
    return mpdd_Rgemm_host_ex(h, None, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C,
                              ldc, _entry="mpdd_Rgemm_host")


def mpdd_Rgemm_host_ex(h, opts, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                       _entry="mpdd_Rgemm_host_ex"):
    """As mpdd_Rgemm_host with explicit options (an mpdd_opts, a dict of its
    fields, or None)."""
    a, bt = _dd(alpha), _dd(beta)
    ext = _gemm_extents(transa, transb, m, n, k, lda, ldb, ldc)
    ab, ct = _touches(ext, _dd_zero(a), _dd_one(bt), k, m, n)
    ea, eb, ec = ext if ext else (0, 0, 0)
    args = (_flag(transa), _flag(transb), m, n, k, a, _host_pairs(A, ea if ab else 0, "A"), lda,
            _host_pairs(B, eb if ab else 0, "B"), ldb, bt, _host_pairs(C, ec if ct else 0, "C"),
            ldc)
    if _entry == "mpdd_Rgemm_host":
        return load().mpdd_Rgemm_host(h, *args)
    return load().mpdd_Rgemm_host_ex(h, _opts_ref(opts), *args)


def mpdd_Rsyrk_host(h, uplo, trans, n, k, alpha, A, lda, beta, C, ldc):
    return mpdd_Rsyrk_host_ex(h, None, uplo, trans, n, k, alpha, A, lda, beta, C, ldc,
                              _entry="mpdd_Rsyrk_host")


def mpdd_Rsyrk_host_ex(h, opts, uplo, trans, n, k, alpha, A, lda, beta, C, ldc,
                       _entry="mpdd_Rsyrk_host_ex"):
    a, bt = _dd(alpha), _dd(beta)
    ext = _syrk_extents(uplo, trans, n, k, lda, ldc)
    ab, ct = _touches(ext, _dd_zero(a), _dd_one(bt), k, n, n)
    ea, ec = ext if ext else (0, 0)
    args = (_flag(uplo), _flag(trans), n, k, a, _host_pairs(A, ea if ab else 0, "A"), lda, bt,
            _host_pairs(C, ec if ct else 0, "C"), ldc)
    if _entry == "mpdd_Rsyrk_host":
        return load().mpdd_Rsyrk_host(h, *args)
    return load().mpdd_Rsyrk_host_ex(h, _opts_ref(opts), *args)


def mpdd_ozaki_digit_widths(algo, k, nslices):
    """(first digit width, later digit width) of a split form; raises if none."""
    a, b = ctypes.c_int(), ctypes.c_int()
    info = load().mpdd_ozaki_digit_widths(algo, k, nslices, ctypes.byref(a), ctypes.byref(b))
    if info != 0:
        raise ValueError(f"no exact digit width for algo={algo} k={k} nslices={nslices}: {info}")
    return a.value, b.value


def mpdd_ozaki_crt_exponent(k, nmoduli):
    """Grid width P of the modular split form; raises if none."""
    p = ctypes.c_int()
    info = load().mpdd_ozaki_crt_exponent(k, nmoduli, ctypes.byref(p))
    if info != 0:
        raise ValueError(f"no modular grid for k={k} nmoduli={nmoduli}: {info}")
    return p.value


def mpdd_ozaki_split(h, algo, trans, rows, k, X, ld, nslices, exps, slices, ldq, rows_p,
                     stream=None):
    """Scale exponents (int32 tensor) and slices (int8 / float64 tensor; the
    modular form: int8 residues) of a row operand, see include/mpdd.h.
    Returns info."""
    import torch
    ft = _first(trans)
    nr, nc = (rows, k) if ft == "N" else (k, rows)
    ok = (ft in ("N", "T", "C") and rows >= 0 and k >= 0 and ld >= max(1, nr) and nslices >= 1
          and ldq >= k and ldq % 64 == 0 and rows_p >= rows and rows_p % 64 == 0
          and algo in (MPDD_OZAKI_I8, MPDD_OZAKI_F64, MPDD_OZAKI_CRT))
    px = _planes(X, _extent(nr, nc, ld) if ok else 0, "X")
    pe = _dev(exps, rows if ok else 0, "exps", torch.int32)
    pq = _dev(slices, nslices * rows_p * ldq if ok else 0, "slices",
              torch.float64 if algo == MPDD_OZAKI_F64 else torch.int8)
    return load().mpdd_ozaki_split(h, algo, _flag(trans), rows, k, px[0], px[1], ld, nslices,
                                   pe, pq, ldq, rows_p, _stream(stream))


def mpdd_tile_count():
    return load().mpdd_tile_count()


def mpdd_tile_info(tile_id):
    vals = [ctypes.c_int() for _ in range(4)]
    info = load().mpdd_tile_info(tile_id, *[ctypes.byref(v) for v in vals])
    if info != 0:
        raise ValueError(f"no tile {tile_id}")
    return tuple(v.value for v in vals)


# ---- request server ---------------------------------------------------------------

def mpdd_struct_size(name):
    return load().mpdd_struct_size(name.encode())


def mpdd_clock():
    return load().mpdd_clock()


def mpdd_server_create(h, hbm_budget_bytes, max_inflight, flags=0):
    s = _P()
    info = load().mpdd_server_create(ctypes.byref(s), h, hbm_budget_bytes, max_inflight, flags)
    if info != 0:
        raise RuntimeError(f"mpdd_server_create failed: {info}")
    return s


def mpdd_server_set_fake_rate(s, dd_flops_per_s, group_latency_s):
    return load().mpdd_server_set_fake_rate(s, dd_flops_per_s, group_latency_s)


def make_request(op, flag1, flag2, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, arrival=-1.0,
                 inject=MPDD_INJECT_NONE):
    """An mpdd_request; A, B, C are (hi, lo) pairs of tensors or device pointers
    (B may be (None, None) for Rsyrk)."""
    r = mpdd_request()
    r.op = op
    r.flag1 = _flag(flag1)
    r.flag2 = _flag(flag2)
    r.m, r.n, r.k = m, n, k
    r.alpha, r.beta = _dd(alpha), _dd(beta)
    ea = eb = ec = 0
    if op == MPDD_OP_SYRK:
        ext = _syrk_extents(flag1, flag2, n, k, lda, ldc)
        ab, ct = _touches(ext, _dd_zero(r.alpha), _dd_one(r.beta), k, n, n)
        if ext:
            ea, ec = ext
    else:
        ext = _gemm_extents(flag1, flag2, m, n, k, lda, ldb, ldc)
        ab, ct = _touches(ext, _dd_zero(r.alpha), _dd_one(r.beta), k, m, n)
        if ext:
            ea, eb, ec = ext
    pa = _planes(A, ea if ab else 0, "A")
    pb = _planes(B, eb if ab else 0, "B")
    pc = _planes(C, ec if ct else 0, "C")
    r.A_hi, r.A_lo, r.lda = pa[0], pa[1], lda
    r.B_hi, r.B_lo, r.ldb = pb[0], pb[1], ldb
    r.C_hi, r.C_lo, r.ldc = pc[0], pc[1], ldc
    r.arrival = arrival
    r.inject = inject
    return r


def mpdd_server_submit(s, req):
    t = ctypes.c_uint64()
    info = load().mpdd_server_submit(s, ctypes.byref(req), ctypes.byref(t))
    if info != 0:
        raise RuntimeError(f"mpdd_server_submit failed: {info}")
    return t.value


def prepared_submit(s):
    """A submit function for server s with its ticket buffer marshalled once:
    submit(req) -> ticket (req from make_request)."""
    t = ctypes.c_uint64()
    tref = ctypes.byref(t)
    fn = load().mpdd_server_submit

    def submit(req):
        info = fn(s, ctypes.byref(req), tref)
        if info != 0:
            raise RuntimeError(f"mpdd_server_submit failed: {info}")
        return t.value
    return submit


def mpdd_server_wait(s, ticket):
    """(info, timing dict) of a request; blocks until it completes."""
    info = ctypes.c_int()
    t = mpdd_timing()
    rc = load().mpdd_server_wait(s, ticket, ctypes.byref(info), ctypes.byref(t))
    if rc != 0:
        raise ValueError(f"mpdd_server_wait: unknown ticket {ticket}")
    return info.value, {f: getattr(t, f) for f, _ in mpdd_timing._fields_}


def mpdd_server_poll(s, ticket):
    d = ctypes.c_int()
    rc = load().mpdd_server_poll(s, ticket, ctypes.byref(d))
    if rc != 0:
        raise ValueError(f"mpdd_server_poll: unknown ticket {ticket}")
    return bool(d.value)


def mpdd_server_get_stats(s):
    st = mpdd_server_stats()
    load().mpdd_server_get_stats(s, ctypes.byref(st))
    return {f: getattr(st, f) for f, _ in mpdd_server_stats._fields_}


def mpdd_server_destroy(s):
    return load().mpdd_server_destroy(s)

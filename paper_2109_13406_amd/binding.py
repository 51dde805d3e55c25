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

MPDD_ERR_HIP = -1
MPDD_ERR_ALLOC = -2
MPDD_ERR_BUDGET = -3
MPDD_ERR_SHUTDOWN = -4
MPDD_ERR_UNSUPPORTED = -5
MPDD_ERR_HANDLE = -6
MPDD_ERR_ARG = -7


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
    "mpdd_Rpotrf": (ctypes.c_int, [_P, _C, _I, _P, _P, _I, ctypes.POINTER(_I), _P]),
    "mpdd_Rpotrf_nb": (ctypes.c_int, [_P, _C, _I, _P, _P, _I, _I, ctypes.POINTER(_I), _P]),
    "mpdd_ozaki_digit_widths": (ctypes.c_int, [ctypes.c_int, _I, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_int)]),
    "mpdd_ozaki_split": (ctypes.c_int, [_P, ctypes.c_int, _C, _I, _I, _P, _P, _I, ctypes.c_int,
                                        _P, _P, _I, _I, _P]),
    "mpdd_Rgemm_host": (ctypes.c_int, [_P, _C, _C, _I, _I, _I, mpdd_dd, _P, _I, _P, _I, mpdd_dd,
                                       _P, _I]),
    "mpdd_Rsyrk_host": (ctypes.c_int, [_P, _C, _C, _I, _I, mpdd_dd, _P, _I, mpdd_dd, _P, _I]),
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


def mpdd_Rgemm(h, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    """A, B, C: (hi, lo) pairs of tensors or device pointers.  Returns info."""
    return load().mpdd_Rgemm(h, _flag(transa), _flag(transb), m, n, k, _dd(alpha), _ptr(A[0]),
                             _ptr(A[1]), lda, _ptr(B[0]), _ptr(B[1]), ldb, _dd(beta), _ptr(C[0]),
                             _ptr(C[1]), ldc, _stream(stream))


def mpdd_Rgemm_ex(h, opts, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                  stream=None):
    o = opts if opts is None or isinstance(opts, mpdd_opts) else _opts(**opts)
    return load().mpdd_Rgemm_ex(h, ctypes.byref(o) if o is not None else None, _flag(transa),
                                _flag(transb), m, n, k, _dd(alpha), _ptr(A[0]), _ptr(A[1]), lda,
                                _ptr(B[0]), _ptr(B[1]), ldb, _dd(beta), _ptr(C[0]), _ptr(C[1]),
                                ldc, _stream(stream))


def mpdd_Cgemm(h, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    """A, B, C: 4-tuples (re.hi, re.lo, im.hi, im.lo) of tensors or device
    pointers.  Returns info."""
    return load().mpdd_Cgemm(h, _flag(transa), _flag(transb), m, n, k, _ddc(alpha),
                             *map(_ptr, A), lda, *map(_ptr, B), ldb, _ddc(beta), *map(_ptr, C),
                             ldc, _stream(stream))


def mpdd_Cgemm_ex(h, opts, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                  stream=None):
    o = opts if opts is None or isinstance(opts, mpdd_opts) else _opts(**opts)
    return load().mpdd_Cgemm_ex(h, ctypes.byref(o) if o is not None else None, _flag(transa),
                                _flag(transb), m, n, k, _ddc(alpha), *map(_ptr, A), lda,
                                *map(_ptr, B), ldb, _ddc(beta), *map(_ptr, C), ldc,
                                _stream(stream))


def _qd(x):
    if isinstance(x, mpdd_qd):
        return x
    if isinstance(x, (int, float)):
        x = (float(x), 0.0, 0.0, 0.0)
    return mpdd_qd((ctypes.c_double * 4)(*[float(v) for v in x]))


def mpdd_Qgemm(h, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    """Quad-double Rgemm.  A, B, C: 4-tuples of planes (x0..x3) as tensors or
    device pointers; alpha, beta: 4-tuples of floats.  Returns info."""
    return load().mpdd_Qgemm(h, _flag(transa), _flag(transb), m, n, k, _qd(alpha),
                             *map(_ptr, A), lda, *map(_ptr, B), ldb, _qd(beta), *map(_ptr, C),
                             ldc, _stream(stream))


def mpdd_Rpotrf(h, uplo, n, A, lda, nb=0, stream=None):
    """A: (hi, lo) pair of tensors or device pointers.  Returns (rc, info):
    rc = 0 or MPDD_ERR_*, info = LAPACK's info."""
    info = _I(0)
    rc = load().mpdd_Rpotrf_nb(h, _flag(uplo), n, _ptr(A[0]), _ptr(A[1]), lda, nb,
                               ctypes.byref(info), _stream(stream))
    return rc, info.value


def mpdd_Rsyrk(h, uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream=None):
    return load().mpdd_Rsyrk(h, _flag(uplo), _flag(trans), n, k, _dd(alpha), _ptr(A[0]),
                             _ptr(A[1]), lda, _dd(beta), _ptr(C[0]), _ptr(C[1]), ldc,
                             _stream(stream))


def mpdd_Rsyrk_ex(h, opts, uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream=None):
    o = opts if opts is None or isinstance(opts, mpdd_opts) else _opts(**opts)
    return load().mpdd_Rsyrk_ex(h, ctypes.byref(o) if o is not None else None, _flag(uplo),
                                _flag(trans), n, k, _dd(alpha), _ptr(A[0]), _ptr(A[1]), lda,
                                _dd(beta), _ptr(C[0]), _ptr(C[1]), ldc, _stream(stream))


def _host_pairs(x):
    """Pointer to an interleaved {hi, lo} host array: a numpy float64 array of
    shape (..., 2) / length 2*count, or None."""
    if x is None:
        return None
    import numpy as np
    assert x.dtype == np.float64 and x.flags.c_contiguous
    return x.ctypes.data


def mpdd_Rgemm_host(h, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    """MPBLAS-shaped Rgemm on host dd_real arrays (numpy float64, {hi, lo}
    interleaved).  Synchronous; returns info."""
    return load().mpdd_Rgemm_host(h, _flag(transa), _flag(transb), m, n, k, _dd(alpha),
                                  _host_pairs(A), lda, _host_pairs(B), ldb, _dd(beta),
                                  _host_pairs(C), ldc)


def mpdd_Rsyrk_host(h, uplo, trans, n, k, alpha, A, lda, beta, C, ldc):
    return load().mpdd_Rsyrk_host(h, _flag(uplo), _flag(trans), n, k, _dd(alpha),
                                  _host_pairs(A), lda, _dd(beta), _host_pairs(C), ldc)


def mpdd_ozaki_digit_widths(algo, k, nslices):
    """(first digit width, later digit width) of a split form; raises if none."""
    a, b = ctypes.c_int(), ctypes.c_int()
    info = load().mpdd_ozaki_digit_widths(algo, k, nslices, ctypes.byref(a), ctypes.byref(b))
    if info != 0:
        raise ValueError(f"no exact digit width for algo={algo} k={k} nslices={nslices}: {info}")
    return a.value, b.value


def mpdd_ozaki_split(h, algo, trans, rows, k, X, ld, nslices, exps, slices, ldq, rows_p,
                     stream=None):
    """Scale exponents (int32 tensor) and slices (int8 / float64 tensor) of a row
    operand, see include/mpdd.h.  Returns info."""
    return load().mpdd_ozaki_split(h, algo, _flag(trans), rows, k, _ptr(X[0]), _ptr(X[1]), ld,
                                   nslices, _ptr(exps), _ptr(slices), ldq, rows_p,
                                   _stream(stream))


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
    r.A_hi, r.A_lo, r.lda = _ptr(A[0]), _ptr(A[1]), lda
    r.B_hi, r.B_lo, r.ldb = _ptr(B[0]), _ptr(B[1]), ldb
    r.C_hi, r.C_lo, r.ldc = _ptr(C[0]), _ptr(C[1]), ldc
    r.arrival = arrival
    r.inject = inject
    return r


def mpdd_server_submit(s, req):
    t = ctypes.c_uint64()
    info = load().mpdd_server_submit(s, ctypes.byref(req), ctypes.byref(t))
    if info != 0:
        raise RuntimeError(f"mpdd_server_submit failed: {info}")
    return t.value


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

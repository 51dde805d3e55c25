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

MPDD_ERR_HIP = -1
MPDD_ERR_ALLOC = -2
MPDD_ERR_BUDGET = -3
MPDD_ERR_SHUTDOWN = -4
MPDD_ERR_UNSUPPORTED = -5
MPDD_ERR_HANDLE = -6
MPDD_ERR_ARG = -7


class mpdd_dd(ctypes.Structure):
    _fields_ = [("hi", ctypes.c_double), ("lo", ctypes.c_double)]


class mpdd_opts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int), ("nslices", ctypes.c_int), ("tile_id", ctypes.c_int),
                ("splitk", ctypes.c_int)]


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


def mpdd_Rsyrk(h, uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream=None):
    return load().mpdd_Rsyrk(h, _flag(uplo), _flag(trans), n, k, _dd(alpha), _ptr(A[0]),
                             _ptr(A[1]), lda, _dd(beta), _ptr(C[0]), _ptr(C[1]), ldc,
                             _stream(stream))


def mpdd_Rsyrk_ex(h, opts, uplo, trans, n, k, alpha, A, lda, beta, C, ldc, stream=None):
    o = opts if opts is None or isinstance(opts, mpdd_opts) else _opts(**opts)
    return load().mpdd_Rsyrk_ex(h, ctypes.byref(o) if o is not None else None, _flag(uplo),
                                _flag(trans), n, k, _dd(alpha), _ptr(A[0]), _ptr(A[1]), lda,
                                _dd(beta), _ptr(C[0]), _ptr(C[1]), ldc, _stream(stream))


def mpdd_tile_count():
    return load().mpdd_tile_count()


def mpdd_tile_info(tile_id):
    vals = [ctypes.c_int() for _ in range(4)]
    info = load().mpdd_tile_info(tile_id, *[ctypes.byref(v) for v in vals])
    if info != 0:
        raise ValueError(f"no tile {tile_id}")
    return tuple(v.value for v in vals)

"""CPU oracle for the double-double MPBLAS / MPLAPACK path -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It loads oracle/liboracle.so (plain C: dd_oracle.c for
Rgemm / Rsyrk, ozaki_oracle.c for the split form, cdd_oracle.c for the
complex Cgemm, potrf_oracle.c for the Cholesky Rpotrf, qd_oracle.c for the
quad-double Rgemm) and exposes
numpy-facing wrappers.  The modular (Chinese-remainder) split form has its
oracle in oracle/crt.py: Python integers and numpy, small sizes.  It never
imports, links or calls the GPU library.

Matrices are passed as pairs (hi, lo) of float64 numpy arrays holding the
column-major storage: a matrix with `rows` rows, `cols` columns and leading
dimension ld is the flat array element [i + j*ld].  Use
`workloads.colmajor(...)` shapes, or numpy arrays in Fortran order.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class _DD(ctypes.Structure):
    _fields_ = [("hi", ctypes.c_double), ("lo", ctypes.c_double)]


def _dd(x):
    if isinstance(x, _DD):
        return x
    hi, lo = (x, 0.0) if np.isscalar(x) else x
    return _DD(float(hi), float(lo))


_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64
_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)


def load(path=None):
    """Load (building first if missing) and return the oracle library."""
    global _LIB
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _LIB is None:
        lib = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(lib):
            _build.build()
        _LIB = _bind(ctypes.CDLL(lib))
    return _LIB


def _bind(lib):
    c = ctypes.c_char_p
    lib.oracle_Rgemm.argtypes = [c, c, _I64, _I64, _I64, _DD, _D, _D, _I64, _D, _D, _I64,
                                 _DD, _D, _D, _I64]
    lib.oracle_Rgemm.restype = ctypes.c_int
    lib.oracle_Rgemm_entries.argtypes = [c, c, _I64, _I64, _I64, _DD, _D, _D, _I64, _D, _D,
                                         _I64, _DD, _D, _D, _I64, _I64, _I64P, _I64P, _D, _D]
    lib.oracle_Rgemm_entries.restype = ctypes.c_int
    lib.oracle_Rsyrk.argtypes = [c, c, _I64, _I64, _DD, _D, _D, _I64, _DD, _D, _D, _I64]
    lib.oracle_Rsyrk.restype = ctypes.c_int
    lib.oracle_Rsyrk_entries.argtypes = [c, c, _I64, _I64, _DD, _D, _D, _I64, _DD, _D, _D,
                                         _I64, _I64, _I64P, _I64P, _D, _D]
    lib.oracle_Rsyrk_entries.restype = ctypes.c_int
    for f in ("oracle_two_sum", "oracle_two_prod"):
        getattr(lib, f).argtypes = [ctypes.c_double, ctypes.c_double, _D, _D]
        getattr(lib, f).restype = None
    for f in ("oracle_dd_add", "oracle_dd_mul"):
        getattr(lib, f).argtypes = [ctypes.c_double] * 4 + [_D, _D]
        getattr(lib, f).restype = None
    lib.oracle_ozaki_split.argtypes = [_I64, _I64, _D, _D, _I64, _I64, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, _I32P, _I32P]
    lib.oracle_ozaki_split.restype = ctypes.c_int
    lib.oracle_ozaki_Rgemm.argtypes = [c, c, _I64, _I64, _I64, _DD, _D, _D, _I64, _D, _D,
                                       _I64, _DD, _D, _D, _I64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int]
    lib.oracle_ozaki_Rgemm.restype = ctypes.c_int
    lib.oracle_Cgemm.argtypes = [c, c, _I64, _I64, _I64, _D, _D, _D, _D, _D, _I64, _D, _D, _D,
                                 _D, _I64, _D, _D, _D, _D, _D, _I64]
    lib.oracle_Cgemm.restype = ctypes.c_int
    lib.oracle_Rpotrf.argtypes = [c, _I64, _D, _D, _I64]
    lib.oracle_Rpotrf.restype = ctypes.c_int64
    lib.oracle_dd_div.argtypes = [ctypes.c_double] * 4 + [_D, _D]
    lib.oracle_dd_div.restype = None
    lib.oracle_dd_sqrt.argtypes = [ctypes.c_double] * 2 + [_D, _D]
    lib.oracle_dd_sqrt.restype = None
    _P4 = _D * 4
    lib.oracle_Qgemm.argtypes = [c, c, _I64, _I64, _I64, _D, _P4, _I64, _P4, _I64, _D, _P4, _I64]
    lib.oracle_Qgemm.restype = ctypes.c_int
    lib.oracle_qd_round_sum.argtypes = [_I64, _D, _D]
    lib.oracle_qd_round_sum.restype = None
    return lib


def _p(a):
    """Pointer to a float64 array (None allowed)."""
    if a is None:
        return None
    assert a.dtype == np.float64 and (a.flags.c_contiguous or a.flags.f_contiguous)
    return a.ctypes.data_as(_D)


def _flag(s):
    return s.encode() if isinstance(s, str) else s


# ---- primitives -------------------------------------------------------------

def two_sum(a, b, lib=None):
    lib = lib or load()
    s, e = ctypes.c_double(), ctypes.c_double()
    lib.oracle_two_sum(a, b, ctypes.byref(s), ctypes.byref(e))
    return s.value, e.value


def two_prod(a, b, lib=None):
    lib = lib or load()
    s, e = ctypes.c_double(), ctypes.c_double()
    lib.oracle_two_prod(a, b, ctypes.byref(s), ctypes.byref(e))
    return s.value, e.value


def dd_add(x, y, lib=None):
    lib = lib or load()
    s, e = ctypes.c_double(), ctypes.c_double()
    lib.oracle_dd_add(x[0], x[1], y[0], y[1], ctypes.byref(s), ctypes.byref(e))
    return s.value, e.value


def dd_mul(x, y, lib=None):
    lib = lib or load()
    s, e = ctypes.c_double(), ctypes.c_double()
    lib.oracle_dd_mul(x[0], x[1], y[0], y[1], ctypes.byref(s), ctypes.byref(e))
    return s.value, e.value


def dd_div(x, y, lib=None):
    lib = lib or load()
    s, e = ctypes.c_double(), ctypes.c_double()
    lib.oracle_dd_div(x[0], x[1], y[0], y[1], ctypes.byref(s), ctypes.byref(e))
    return s.value, e.value


def dd_sqrt(x, lib=None):
    lib = lib or load()
    s, e = ctypes.c_double(), ctypes.c_double()
    lib.oracle_dd_sqrt(x[0], x[1], ctypes.byref(s), ctypes.byref(e))
    return s.value, e.value


def _planes4(P):
    if P is None or P[0] is None:
        return (_D * 4)(None, None, None, None)
    return (_D * 4)(*[_p(x) for x in P])


def qgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, lib=None):
    """In-place oracle quad-double Rgemm: A, B, C are 4-tuples of planes
    (x0, x1, x2, x3); alpha, beta 4-tuples of floats.  Every entry is the exact
    result rounded to a qd.  Returns info."""
    lib = lib or load()
    al = np.asarray(alpha, dtype=np.float64)
    be = np.asarray(beta, dtype=np.float64)
    return lib.oracle_Qgemm(_flag(transa), _flag(transb), m, n, k, _p(al), _planes4(A), lda,
                            _planes4(B), ldb, _p(be), _planes4(C), ldc)


def qd_round_sum(terms, lib=None):
    """Round the exact sum of binary64 terms to a qd (x0, x1, x2, x3)."""
    lib = lib or load()
    t = np.ascontiguousarray(terms, dtype=np.float64)
    q = np.zeros(4)
    lib.oracle_qd_round_sum(t.size, _p(t), _p(q))
    return tuple(float(x) for x in q)


def rpotrf(uplo, n, A, lda, lib=None):
    """In-place oracle Rpotrf on a numpy (hi, lo) pair; returns LAPACK's info."""
    lib = lib or load()
    return int(lib.oracle_Rpotrf(_flag(uplo), n, _p(A[0]), _p(A[1]), lda))


# ---- level 3 ------------------------------------------------------------------

def rgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, lib=None):
    """In-place oracle Rgemm on numpy (hi, lo) pairs; returns info.

    A, B may be (None, None) when alpha == 0 or k == 0, as in BLAS."""
    lib = lib or load()
    return lib.oracle_Rgemm(_flag(transa), _flag(transb), m, n, k, _dd(alpha),
                            _p(A[0]), _p(A[1]), lda, _p(B[0]), _p(B[1]), ldb,
                            _dd(beta), _p(C[0]), _p(C[1]), ldc)


def _cdd(x):
    """complex dd scalar ((re_hi, re_lo), (im_hi, im_lo)), or a Python complex
    (binary64 parts) -> float64[4] = re.hi, re.lo, im.hi, im.lo."""
    if isinstance(x, complex) or np.isscalar(x):
        x = complex(x)
        return np.array([x.real, 0.0, x.imag, 0.0])
    (rh, rl), (ih, il) = x
    return np.array([rh, rl, ih, il], dtype=np.float64)


def cgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, lib=None):
    """In-place oracle Cgemm; A, B, C are 4-tuples of planes (re.hi, re.lo,
    im.hi, im.lo); A, B may be 4-tuples of None when alpha == 0 or k == 0.
    Returns info."""
    lib = lib or load()
    al, be = _cdd(alpha), _cdd(beta)
    return lib.oracle_Cgemm(_flag(transa), _flag(transb), m, n, k, _p(al), *map(_p, A), lda,
                            *map(_p, B), ldb, _p(be), *map(_p, C), ldc)


def rsyrk(uplo, trans, n, k, alpha, A, lda, beta, C, ldc, lib=None):
    """In-place oracle Rsyrk on numpy (hi, lo) pairs; returns info."""
    lib = lib or load()
    return lib.oracle_Rsyrk(_flag(uplo), _flag(trans), n, k, _dd(alpha),
                            _p(A[0]), _p(A[1]), lda, _dd(beta), _p(C[0]), _p(C[1]), ldc)


def _entries_common(ii, jj):
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    out_h = np.empty(ii.shape[0])
    out_l = np.empty(ii.shape[0])
    return ii, jj, out_h, out_l


def rgemm_entries(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ii, jj,
                  lib=None):
    """Selected entries (ii[t], jj[t]) of the Rgemm result; C is not written.

    Returns (hi, lo) arrays."""
    lib = lib or load()
    ii, jj, oh, ol = _entries_common(ii, jj)
    info = lib.oracle_Rgemm_entries(
        _flag(transa), _flag(transb), m, n, k, _dd(alpha), _p(A[0]), _p(A[1]), lda,
        _p(B[0]), _p(B[1]), ldb, _dd(beta), _p(C[0]), _p(C[1]), ldc, ii.shape[0],
        ii.ctypes.data_as(_I64P), jj.ctypes.data_as(_I64P), _p(oh), _p(ol))
    if info != 0:
        raise ValueError(f"oracle_Rgemm_entries info={info}")
    return oh, ol


def rsyrk_entries(uplo, trans, n, k, alpha, A, lda, beta, C, ldc, ii, jj, lib=None):
    """Selected entries of the Rsyrk result (all in the uplo triangle)."""
    lib = lib or load()
    ii, jj, oh, ol = _entries_common(ii, jj)
    info = lib.oracle_Rsyrk_entries(
        _flag(uplo), _flag(trans), n, k, _dd(alpha), _p(A[0]), _p(A[1]), lda, _dd(beta),
        _p(C[0]), _p(C[1]), ldc, ii.shape[0], ii.ctypes.data_as(_I64P),
        jj.ctypes.data_as(_I64P), _p(oh), _p(ol))
    if info != 0:
        raise ValueError(f"oracle_Rsyrk_entries info={info}")
    return oh, ol


# ---- split form -----------------------------------------------------------------

INT8_QMAX = 127            # largest int8 digit: later digits are carried into [-128, 127]


def int8_digit_widths(k, nslices):
    """(first, later) digit widths of INT8 slices, or None: 8-bit later
    digits while nslices*k < 2^17, 7-bit ones (|q| <= 64) while
    nslices*k < 2^19, so that every anti-diagonal sum of at most nslices*k
    digit products (each at most 2^(2w-2) in magnitude) stays below 2^31."""
    terms = int(k) * int(nslices)
    if terms < 2 ** 17:
        return 6, 8
    if terms < 2 ** 19:
        return 6, 7
    return None


def fp64_digit_width(k, nslices):
    """Digit width w for FP64 slices: every partial sum of up to nslices*k
    products of two digits (|q| <= 2^(w-1)) stays an integer below 2^53,
    so FP64 accumulation of the slice products is exact."""
    terms = max(1, int(k) * int(nslices))
    lg = (terms - 1).bit_length()          # ceil(log2(terms))
    w = (55 - lg) // 2
    return w - 1, w


def ozaki_split(rows, k, X, sr, sl, nslices, wfirst, w, qmax=0, lib=None):
    """Scale exponents (rows,) and digits (nslices, rows, k) of a row operand
    whose element (r, l) is X[r*sr + l*sl] (flat hi/lo arrays); qmax > 0
    carries the digits after the first into [.., qmax]."""
    lib = lib or load()
    exps = np.zeros(rows, dtype=np.int32)
    digs = np.zeros((nslices, rows, k), dtype=np.int32)
    info = lib.oracle_ozaki_split(rows, k, _p(X[0]), _p(X[1]), sr, sl, nslices, wfirst, w, qmax,
                                  exps.ctypes.data_as(_I32P), digs.ctypes.data_as(_I32P))
    if info != 0:
        raise ValueError("oracle_ozaki_split failed")
    return exps, digs


def ozaki_rgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nslices,
                wfirst, w, qmax=0, lib=None):
    lib = lib or load()
    return lib.oracle_ozaki_Rgemm(_flag(transa), _flag(transb), m, n, k, _dd(alpha),
                                  _p(A[0]), _p(A[1]), lda, _p(B[0]), _p(B[1]), ldb,
                                  _dd(beta), _p(C[0]), _p(C[1]), ldc, nslices, wfirst, w, qmax)

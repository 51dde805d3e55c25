"""The C-ABI library without a GPU: it loads, exports every symbol that
include/*.h declares, and its host-side argument checks report the BLAS
argument positions (checked before the handle, so no HIP call is made)."""
import ctypes
import os
import re

import pytest

import pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(inc, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w \*]*?\b(mpdd_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2109_13406_amd import binding
    return binding.load()


def test_header_declares_entry_points():
    names = _declared_functions()
    for must in ("mpdd_create", "mpdd_destroy", "mpdd_Rgemm", "mpdd_Rsyrk", "mpdd_Rgemm_ex"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2109_13406_amd import binding
    for name in binding.SIGNATURES:
        assert name in _declared_functions(), name


def _gemm(lib, transa="N", transb="N", m=2, n=2, k=2, lda=None, ldb=None, ldc=None):
    from paper_2109_13406_amd import binding as b
    nra = m if transa.upper() == "N" else k
    nrb = k if transb.upper() == "N" else n
    lda = max(1, nra) if lda is None else lda
    ldb = max(1, nrb) if ldb is None else ldb
    ldc = max(1, m) if ldc is None else ldc
    return lib.mpdd_Rgemm(None, transa.encode(), transb.encode(), m, n, k, b.mpdd_dd(1.0, 0.0),
                          None, None, lda, None, None, ldb, b.mpdd_dd(0.5, 0.0), None, None, ldc,
                          None)


def _syrk(lib, uplo="U", trans="N", n=2, k=2, lda=None, ldc=None):
    from paper_2109_13406_amd import binding as b
    nra = n if trans.upper() == "N" else k
    lda = max(1, nra) if lda is None else lda
    ldc = max(1, n) if ldc is None else ldc
    return lib.mpdd_Rsyrk(None, uplo.encode(), trans.encode(), n, k, b.mpdd_dd(1.0, 0.0), None,
                          None, lda, b.mpdd_dd(0.5, 0.0), None, None, ldc, None)


def test_info_codes_match_blas_positions(lib):
    from paper_2109_13406_amd import binding as b
    pos = pins.read_arg_positions()
    H = b.MPDD_ERR_HANDLE          # valid arguments reach the handle check
    g = lambda **kw: _gemm(lib, **kw)
    s = lambda **kw: _syrk(lib, **kw)
    assert g() == H
    for t in "NnTtCc":
        assert g(transa=t) == H and g(transb=t) == H
    assert g(transa="X") == pos[("gemm", "transa")]
    assert g(transb="q") == pos[("gemm", "transb")]
    assert g(transa="X", m=-1) == pos[("gemm", "transa")]
    assert g(m=-1) == pos[("gemm", "m")]
    assert g(n=-1) == pos[("gemm", "n")]
    assert g(k=-1) == pos[("gemm", "k")]
    assert g(m=5, lda=4) == pos[("gemm", "lda")]
    assert g(transa="T", m=5, k=3, lda=3) == H
    assert g(transa="T", m=3, k=5, lda=4) == pos[("gemm", "lda")]
    assert g(k=5, ldb=4) == pos[("gemm", "ldb")]
    assert g(transb="T", n=5, k=3, ldb=4) == pos[("gemm", "ldb")]
    assert g(m=5, lda=5, ldc=4) == pos[("gemm", "ldc")]
    assert g(m=0, lda=0) == pos[("gemm", "lda")]
    assert s() == H
    assert s(uplo="x") == pos[("syrk", "uplo")]
    assert s(trans="z") == pos[("syrk", "trans")]
    assert s(trans="c") == H
    assert s(n=-1) == pos[("syrk", "n")]
    assert s(k=-1) == pos[("syrk", "k")]
    assert s(n=5, lda=4) == pos[("syrk", "lda")]
    assert s(trans="T", n=3, k=5, lda=4) == pos[("syrk", "lda")]
    assert s(n=5, lda=5, ldc=4) == pos[("syrk", "ldc")]


def test_null_flag_is_invalid(lib):
    from paper_2109_13406_amd import binding as b
    info = lib.mpdd_Rgemm(None, None, b"N", 1, 1, 1, b.mpdd_dd(1.0, 0.0), None, None, 1, None,
                          None, 1, b.mpdd_dd(0.0, 0.0), None, None, 1, None)
    assert info == 1


def test_tile_table(lib):
    from paper_2109_13406_amd import binding as b
    n = b.mpdd_tile_count()
    assert n >= 1
    for i in range(n):
        bm, bn, bk, threads = b.mpdd_tile_info(i)
        assert bm > 0 and bn > 0 and bk > 0 and threads % 64 == 0
    with pytest.raises(ValueError):
        b.mpdd_tile_info(n)


def test_destroy_null_handle(lib):
    from paper_2109_13406_amd import binding as b
    assert lib.mpdd_destroy(None) == b.MPDD_ERR_HANDLE


def test_cgemm_info_codes_before_handle(lib):
    """Cgemm checks ZGEMM's argument positions on the host before anything
    else; valid arguments reach the handle check."""
    from paper_2109_13406_amd import binding as b
    pos = pins.read_arg_positions()
    one = b.mpdd_ddc(b.mpdd_dd(1.0, 0.0), b.mpdd_dd(0.0, 0.0))
    N4 = (None,) * 4

    def c(ta="N", tb="N", m=2, n=2, k=2, lda=None, ldb=None, ldc=None):
        lda = lda if lda is not None else max(1, m if ta.upper() == "N" else k)
        ldb = ldb if ldb is not None else max(1, k if tb.upper() == "N" else n)
        ldc = ldc if ldc is not None else max(1, m)
        return lib.mpdd_Cgemm(None, ta.encode(), tb.encode(), m, n, k, one, *N4, lda, *N4, ldb,
                              one, *N4, ldc, None)
    H = b.MPDD_ERR_HANDLE
    for t in "NnTtCc":
        assert c(ta=t) == H and c(tb=t) == H
    assert c(ta="X") == pos[("gemm", "transa")]
    assert c(tb="q") == pos[("gemm", "transb")]
    assert c(m=-1) == pos[("gemm", "m")]
    assert c(n=-1) == pos[("gemm", "n")]
    assert c(k=-1) == pos[("gemm", "k")]
    assert c(ta="C", m=3, k=2, lda=1) == pos[("gemm", "lda")]
    assert c(tb="C", n=3, k=2, ldb=2) == pos[("gemm", "ldb")]
    assert c(m=3, ldc=2) == pos[("gemm", "ldc")]


def test_struct_sizes_match_binding(lib):
    from paper_2109_13406_amd import binding as b
    for name in ("mpdd_dd", "mpdd_ddc", "mpdd_qd", "mpdd_opts", "mpdd_request", "mpdd_timing",
                 "mpdd_server_stats"):
        assert lib.mpdd_struct_size(name.encode()) == ctypes.sizeof(getattr(b, name)), name


def test_potrf_argument_errors_before_handle(lib):
    """Rpotrf reports LAPACK's negative argument positions in *info (return
    value 0) before looking at the handle; valid arguments reach the handle
    check; a NULL info pointer is rejected."""
    from paper_2109_13406_amd import binding as b
    info = ctypes.c_int64(99)

    def p(uplo, n, lda, nb=0):
        info.value = 99
        rc = lib.mpdd_Rpotrf_nb(None, uplo, n, None, None, lda, nb, ctypes.byref(info), None)
        return rc, info.value
    assert p(b"X", 4, 4) == (0, -1)
    assert p(b"l", -1, 4) == (0, -2)
    assert p(b"U", 4, 3) == (0, -4)
    assert p(b"u", 0, 0) == (0, -4)
    assert p(b"L", 4, 4) == (b.MPDD_ERR_HANDLE, 0)
    assert lib.mpdd_Rpotrf(None, b"L", 4, None, None, 4, None, None) == b.MPDD_ERR_ARG


def test_qgemm_info_codes_before_handle(lib):
    from paper_2109_13406_amd import binding as b
    pos = pins.read_arg_positions()
    one = b._qd((1.0, 0.0, 0.0, 0.0))
    N4 = (None,) * 4

    def q(ta="N", tb="N", m=2, n=2, k=2, lda=None, ldb=None, ldc=None):
        lda = lda if lda is not None else max(1, m if ta.upper() == "N" else k)
        ldb = ldb if ldb is not None else max(1, k if tb.upper() == "N" else n)
        ldc = ldc if ldc is not None else max(1, m)
        return lib.mpdd_Qgemm(None, ta.encode(), tb.encode(), m, n, k, one, *N4, lda, *N4, ldb,
                              one, *N4, ldc, None)
    H = b.MPDD_ERR_HANDLE
    assert q() == H and q(ta="t", tb="C") == H
    assert q(ta="X") == pos[("gemm", "transa")]
    assert q(tb="z") == pos[("gemm", "transb")]
    assert q(m=-1) == pos[("gemm", "m")]
    assert q(n=-1) == pos[("gemm", "n")]
    assert q(k=-1) == pos[("gemm", "k")]
    assert q(m=3, lda=2) == pos[("gemm", "lda")]
    assert q(k=3, ldb=2) == pos[("gemm", "ldb")]
    assert q(m=3, lda=3, ldc=2) == pos[("gemm", "ldc")]


def test_int8_digit_width_guard_is_strict():
    """INT8 split form: every anti-diagonal sum is at most nslices*k*2^(2w-2)
    in magnitude and must stay below 2^31: 8-bit later digits while
    nslices*k < 2^17, 7-bit ones while nslices*k < 2^19; s*k = 2^19 is
    rejected, one less is accepted, and the widths follow the oracle's rule."""
    import oracle
    from paper_2109_13406_amd import binding as b
    wf, w = ctypes.c_int(), ctypes.c_int()
    lib = b.load()
    for s, k, ok, want in ((16, 1 << 15, False, None), (8, 1 << 16, False, None),
                           (1, 1 << 19, False, None), (16, (1 << 15) - 1, True, (6, 7)),
                           (1, (1 << 19) - 1, True, (6, 7)), (16, 1 << 13, True, (6, 7)),
                           (16, (1 << 13) - 1, True, (6, 8)), (13, 8192, True, (6, 8)),
                           (1, (1 << 17) - 1, True, (6, 8)), (1, 1 << 17, True, (6, 7))):
        rc = lib.mpdd_ozaki_digit_widths(b.MPDD_OZAKI_I8, k, s, ctypes.byref(wf), ctypes.byref(w))
        assert (rc == 0) == ok, (s, k, rc)
        assert oracle.int8_digit_widths(k, s) == want
        if not ok:
            assert rc == b.MPDD_ERR_UNSUPPORTED
        else:
            assert (wf.value, w.value) == want, (s, k)


def test_noalloc_info_codes_before_handle(lib):
    """The no-allocation Rgemm checks DGEMM's argument positions on the host
    before anything else, like mpdd_Rgemm_ex; valid arguments reach the
    handle check."""
    from paper_2109_13406_amd import binding as b
    pos = pins.read_arg_positions()

    def g(ta="N", tb="N", m=2, n=2, k=2, lda=None, ldb=None, ldc=None):
        lda = lda if lda is not None else max(1, m if ta.upper() == "N" else k)
        ldb = ldb if ldb is not None else max(1, k if tb.upper() == "N" else n)
        ldc = ldc if ldc is not None else max(1, m)
        return lib.mpdd_Rgemm_noalloc(None, None, ta.encode(), tb.encode(), m, n, k,
                                      b.mpdd_dd(1.0, 0.0), None, None, lda, None, None, ldb,
                                      b.mpdd_dd(0.5, 0.0), None, None, ldc, None)
    assert g() == b.MPDD_ERR_HANDLE
    assert g(ta="x") == pos[("gemm", "transa")]
    assert g(tb="x") == pos[("gemm", "transb")]
    assert g(m=-1) == pos[("gemm", "m")]
    assert g(n=-1) == pos[("gemm", "n")]
    assert g(k=-1) == pos[("gemm", "k")]
    assert g(m=5, lda=4) == pos[("gemm", "lda")]
    assert g(k=5, ldb=4) == pos[("gemm", "ldb")]
    assert g(m=5, lda=5, ldc=4) == pos[("gemm", "ldc")]
    assert b.MPDD_STATIC_SCRATCH_BYTES == 64 << 20
    hdr = open(os.path.join(ROOT, "include", "mpdd.h")).read()
    assert "#define MPDD_STATIC_SCRATCH_BYTES ((size_t)64 << 20)" in hdr
    assert "#define MPDD_ERR_SCRATCH (-8)" in hdr


def test_crt_exponent_matches_the_modular_oracle(lib):
    """The library's grid width P of the modular form (host arithmetic on the
    moduli product) equals the oracle's for every moduli count and a range of
    k, and the same rejections: k >= 2^17, too few moduli, counts outside
    1..32, a null output."""
    from oracle import crt as CRT
    from paper_2109_13406_amd import binding as b
    p = ctypes.c_int()
    for count in range(1, CRT.MAX_MODULI + 1):
        for k in (0, 1, 2, 3, 7, 64, 100, 1000, 2048, 4097, 8192, 65536, 131071):
            want = CRT.exponent(k, count)
            rc = lib.mpdd_ozaki_crt_exponent(k, count, ctypes.byref(p))
            if want is None:
                assert rc == b.MPDD_ERR_UNSUPPORTED, (k, count)
            else:
                assert rc == 0 and p.value == want, (k, count, p.value, want)
    assert lib.mpdd_ozaki_crt_exponent(131072, 32, ctypes.byref(p)) == b.MPDD_ERR_UNSUPPORTED
    for bad in (0, 33):
        assert lib.mpdd_ozaki_crt_exponent(64, bad, ctypes.byref(p)) == b.MPDD_ERR_ARG
    assert lib.mpdd_ozaki_crt_exponent(-1, 10, ctypes.byref(p)) == b.MPDD_ERR_ARG
    assert lib.mpdd_ozaki_crt_exponent(64, 10, None) == b.MPDD_ERR_ARG

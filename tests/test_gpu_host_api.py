"""GPU parity of the MPBLAS-shaped host entry points (dd_real {hi, lo} pairs in
host memory): results equal the oracle's within 8 k 2^-104, the worked example
is exact, beta = 0 ignores NaN in C, padding rows and the opposite triangle
come back bit-identical, and the info codes match the device calls'."""
import numpy as np
import pytest

import oracle
import pins
import workloads as W
from gpu_util import log
from oracle.compare import RATIO_MAX, bits, ratio

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    from paper_2109_13406_amd import binding as b
    assert torch.cuda.is_available()
    handle = b.mpdd_create()
    yield handle
    torch.cuda.synchronize()
    b.mpdd_destroy(handle)


def pairs(pl):
    """(hi, lo) planes -> interleaved {hi, lo} array of shape (n, 2)."""
    return np.ascontiguousarray(np.stack([pl[0], pl[1]], axis=1))


def planes(pr):
    return pr[:, 0].copy(), pr[:, 1].copy()


def test_worked_example_host(h):
    from paper_2109_13406_amd import binding as b
    alpha, beta, v = pins.read_worked_example()
    z = np.zeros(9)
    A = pairs((pins.colmajor(v["A"]), z))
    B = pairs((pins.colmajor(v["B"]), z))
    C = pairs((pins.colmajor(v["C"]), z))
    assert b.mpdd_Rgemm_host(h, "n", "n", 3, 3, 3, alpha, A, 3, B, 3, beta, C, 3) == 0
    assert np.array_equal(C[:, 0], pins.colmajor(v["ANSWER"])) and np.all(C[:, 1] == 0)


@pytest.mark.parametrize("op", W.OPS)
def test_rgemm_host_vs_oracle(h, op):
    from paper_2109_13406_amd import binding as b
    for (m, n, k) in [(97, 131, 77), (1, 1, 1), (130, 65, 200)]:
        for beta_zero in (False, True):
            case = W.gemm_case(1500 + m, op[0], op[1], m, n, k, dist="wide",
                               beta_zero=beta_zero, c_nan=beta_zero)
            O = (case["C"][0].copy(), case["C"][1].copy())
            assert oracle.rgemm(op[0], op[1], m, n, k, case["alpha"], case["A"], case["lda"],
                                case["B"], case["ldb"], case["beta"], O, case["ldc"]) == 0
            C = pairs(case["C"])
            info = b.mpdd_Rgemm_host(h, op[0], op[1], m, n, k, case["alpha"], pairs(case["A"]),
                                     case["lda"], pairs(case["B"]), case["ldb"], case["beta"], C,
                                     case["ldc"])
            assert info == 0
            G = planes(C)
            i, j = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
            idx = (i + j * case["ldc"]).ravel()
            r = ratio(G[0][idx], G[1][idx], O[0][idx], O[1][idx], k)
            assert r <= RATIO_MAX, (op, m, n, k, r)
            rest = np.ones(G[0].shape[0], bool)
            rest[idx] = False
            assert np.array_equal(bits(G[0])[rest], bits(case["C"][0])[rest])
    log(f"PARITY host-pointer Rgemm {op} ok")


@pytest.mark.parametrize("op", W.OPS)
def test_rgemm_host_chunked(h, op):
    """Wide C: several column chunks (ragged last chunk) whose copies overlap
    the products of the chunks before them; with k >= 1024 and op(A) = A the
    first chunk is multiplied in k-slices as A's columns arrive."""
    from paper_2109_13406_amd import binding as b
    for (m, n, k) in [(40, 4100, 50), (33, 1500, 70), (300, 1100, 2100)]:
        case = W.gemm_case(1700 + n, op[0], op[1], m, n, k, dist="wide")
        O = (case["C"][0].copy(), case["C"][1].copy())
        assert oracle.rgemm(op[0], op[1], m, n, k, case["alpha"], case["A"], case["lda"],
                            case["B"], case["ldb"], case["beta"], O, case["ldc"]) == 0
        C = pairs(case["C"])
        assert b.mpdd_Rgemm_host(h, op[0], op[1], m, n, k, case["alpha"], pairs(case["A"]),
                                 case["lda"], pairs(case["B"]), case["ldb"], case["beta"], C,
                                 case["ldc"]) == 0
        G = planes(C)
        i, j = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
        idx = (i + j * case["ldc"]).ravel()
        r = ratio(G[0][idx], G[1][idx], O[0][idx], O[1][idx], k)
        assert r <= RATIO_MAX, (op, m, n, k, r)
        rest = np.ones(G[0].shape[0], bool)
        rest[idx] = False
        assert np.array_equal(bits(G[0])[rest], bits(case["C"][0])[rest])
    log(f"PARITY host-pointer Rgemm chunked {op} ok")


@pytest.mark.parametrize("uplo", "UL")
@pytest.mark.parametrize("trans", "NT")
def test_rsyrk_host_vs_oracle(h, uplo, trans):
    from paper_2109_13406_amd import binding as b
    n, k = 97, 45
    case = W.syrk_case(1600, uplo, trans, n, k, dist="wide")
    O = (case["C"][0].copy(), case["C"][1].copy())
    assert oracle.rsyrk(uplo, trans, n, k, case["alpha"], case["A"], case["lda"], case["beta"], O,
                        case["ldc"]) == 0
    C = pairs(case["C"])
    assert b.mpdd_Rsyrk_host(h, uplo, trans, n, k, case["alpha"], pairs(case["A"]), case["lda"],
                             case["beta"], C, case["ldc"]) == 0
    G = planes(C)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    sel = (i <= j) if uplo == "U" else (i >= j)
    idx = (i + j * case["ldc"])[sel]
    assert ratio(G[0][idx], G[1][idx], O[0][idx], O[1][idx], k) <= RATIO_MAX
    rest = np.ones(G[0].shape[0], bool)
    rest[idx] = False
    assert np.array_equal(bits(G[0])[rest], bits(case["C"][0])[rest])
    assert np.array_equal(bits(G[1])[rest], bits(case["C"][1])[rest])


@pytest.mark.parametrize("op", ["NN", "TN"])
def test_rgemm_host_staged_pieces(h, op):
    """Operands larger than one pinned staging buffer (16 MiB): A and each
    column chunk of C travel in several pieces through the ring, up and
    down; two handles in turn, and a second call that reuses the ring."""
    from paper_2109_13406_amd import binding as b
    m, n, k = 2100, 1100, 800
    case = W.gemm_case(1800, op[0], op[1], m, n, k, dist="wide")
    assert case["C"][0].size * 16 > 2 * (16 << 20)
    O = (case["C"][0].copy(), case["C"][1].copy())
    assert oracle.rgemm(op[0], op[1], m, n, k, case["alpha"], case["A"], case["lda"],
                        case["B"], case["ldb"], case["beta"], O, case["ldc"]) == 0
    i, j = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    idx = (i + j * case["ldc"]).ravel()
    rest = np.ones(O[0].shape[0], bool)
    rest[idx] = False
    h2 = b.mpdd_create()
    try:
        for handle in (h, h2, h):
            C = pairs(case["C"])
            assert b.mpdd_Rgemm_host(handle, op[0], op[1], m, n, k, case["alpha"],
                                     pairs(case["A"]), case["lda"], pairs(case["B"]),
                                     case["ldb"], case["beta"], C, case["ldc"]) == 0
            G = planes(C)
            r = ratio(G[0][idx], G[1][idx], O[0][idx], O[1][idx], k)
            assert r <= RATIO_MAX, (op, r)
            assert np.array_equal(bits(G[0])[rest], bits(case["C"][0])[rest])
    finally:
        b.mpdd_destroy(h2)
    log(f"PARITY host-pointer Rgemm {op} {m}x{n}x{k} through the pinned ring ok")


def test_rsyrk_host_staged_pieces(h):
    from paper_2109_13406_amd import binding as b
    n, k = 1100, 1100
    case = W.syrk_case(1810, "L", "N", n, k, dist="wide")
    O = (case["C"][0].copy(), case["C"][1].copy())
    assert oracle.rsyrk("L", "N", n, k, case["alpha"], case["A"], case["lda"], case["beta"], O,
                        case["ldc"]) == 0
    C = pairs(case["C"])
    assert b.mpdd_Rsyrk_host(h, "L", "N", n, k, case["alpha"], pairs(case["A"]), case["lda"],
                             case["beta"], C, case["ldc"]) == 0
    G = planes(C)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    idx = (i + j * case["ldc"])[i >= j]
    assert ratio(G[0][idx], G[1][idx], O[0][idx], O[1][idx], k) <= RATIO_MAX
    rest = np.ones(G[0].shape[0], bool)
    rest[idx] = False
    assert np.array_equal(bits(G[0])[rest], bits(case["C"][0])[rest])


def test_host_info_codes(h):
    from paper_2109_13406_amd import binding as b
    C = np.zeros((9, 2))
    assert b.mpdd_Rgemm_host(h, "X", "N", 3, 3, 3, 1.0, None, 3, None, 3, 0.0, C, 3) == 1
    assert b.mpdd_Rgemm_host(h, "N", "N", 3, 3, 3, 1.0, None, 2, None, 3, 0.0, C, 3) == 8
    assert b.mpdd_Rsyrk_host(h, "U", "N", 3, 3, 1.0, None, 3, 0.0, C, 2) == 10
    assert b.mpdd_Rgemm_host(h, "N", "N", 0, 3, 3, 1.0, None, 1, None, 3, 0.0, C, 1) == 0


def test_rgemm_host_8192_sampled(h):
    """The benchmarked host-pointer call (8192^3 NN, ld 8195, dd_real pairs in
    pageable host memory, alpha 0.5, beta 0.25, the bench's device-generated
    inputs brought to the host) on 64 sampled entries against the oracle, and
    the padding rows of C untouched."""
    import torch
    from paper_2109_13406_amd import binding as b
    n = 8192
    case = W.gemm_case_device(W.BASE_SEED + 5, "N", "N", n, n, n)
    hp = lambda pl: torch.stack([pl[0], pl[1]], dim=1).cpu().numpy()
    A, B, C = hp(case["A"]), hp(case["B"]), hp(case["C"])
    ld = case["lda"]
    del case
    torch.cuda.empty_cache()
    C0 = C.copy()
    alpha, beta = (0.5, 0.0), (0.25, 0.0)
    assert b.mpdd_Rgemm_host(h, "N", "N", n, n, n, alpha, A, ld, B, ld, beta, C, ld) == 0
    rng = np.random.default_rng(13)
    ii = np.concatenate([rng.integers(0, n, 60), [0, n - 1, 0, n - 1]])
    jj = np.concatenate([rng.integers(0, n, 60), [0, n - 1, n - 1, 0]])
    P = lambda x: (np.ascontiguousarray(x[:, 0]), np.ascontiguousarray(x[:, 1]))
    oh, ol = oracle.rgemm_entries("N", "N", n, n, n, alpha, P(A), ld, P(B), ld, beta, P(C0), ld,
                                  ii, jj)
    idx = ii + jj * ld
    r = ratio(C[idx, 0], C[idx, 1], oh, ol, n)
    log(f"PARITY host-pointer Rgemm {n}^3 NN sampled 64: ratio {r:.4g}")
    assert r <= RATIO_MAX
    pad = (np.arange(n, ld)[:, None] + np.arange(0, n, 97)[None, :] * ld).ravel()
    assert np.array_equal(bits(C[pad, 0]), bits(C0[pad, 0]))
    assert np.array_equal(bits(C[pad, 1]), bits(C0[pad, 1]))


def tight(pl, extent, pad=37):
    """Interleaved pairs of the first `extent` entries of planes `pl`, as a
    view of a larger buffer whose `pad` further pairs hold a NaN sentinel."""
    buf = np.empty((extent + pad, 2))
    buf[:extent] = pairs((pl[0][:extent], pl[1][:extent]))
    buf[extent:] = np.array([0x7FF8DEAD00000001, 0x7FF8DEAD00000002], np.uint64).view(np.float64)
    return buf, buf[:extent]


@pytest.mark.parametrize("op", W.OPS)
def test_rgemm_host_exact_extent(h, op):
    """Arrays sized exactly to their BLAS extent ld*(cols-1) + rows (large
    enough for column chunks and k-slices): the result matches the oracle and
    nothing past any array's extent is written."""
    from paper_2109_13406_amd import binding as b
    m, n, k = 300, 1100, 1090
    case = W.gemm_case(1900, op[0], op[1], m, n, k, dist="wide")
    ra, ca = (m, k) if op[0] == "N" else (k, m)
    rb, cb = (k, n) if op[1] == "N" else (n, k)
    ea = case["lda"] * (ca - 1) + ra
    eb = case["ldb"] * (cb - 1) + rb
    ec = case["ldc"] * (n - 1) + m
    O = (case["C"][0].copy(), case["C"][1].copy())
    assert oracle.rgemm(op[0], op[1], m, n, k, case["alpha"], case["A"], case["lda"],
                        case["B"], case["ldb"], case["beta"], O, case["ldc"]) == 0
    bufs = [tight(case["A"], ea), tight(case["B"], eb), tight(case["C"], ec)]
    before = [x[0].copy() for x in bufs]
    assert b.mpdd_Rgemm_host(h, op[0], op[1], m, n, k, case["alpha"], bufs[0][1], case["lda"],
                             bufs[1][1], case["ldb"], case["beta"], bufs[2][1], case["ldc"]) == 0
    for (full, _), old, e in zip(bufs, before, (ea, eb, ec)):
        assert np.array_equal(bits(full[e:].ravel()), bits(old[e:].ravel())), op
    G = planes(bufs[2][1])
    idx = (np.arange(m)[:, None] + np.arange(n)[None, :] * case["ldc"]).ravel()
    r = ratio(G[0][idx], G[1][idx], O[0][idx], O[1][idx], k)
    assert r <= RATIO_MAX, (op, r)
    rest = np.ones(ec, bool)
    rest[idx] = False
    assert np.array_equal(bits(G[0])[rest], bits(case["C"][0][:ec])[rest])
    log(f"PARITY host-pointer Rgemm {op} exact-extent arrays ratio={r:.3g}")


@pytest.mark.parametrize("trans", ["N", "T"])
def test_rsyrk_host_exact_extent(h, trans):
    from paper_2109_13406_amd import binding as b
    n, k = 260, 300
    case = W.syrk_case(1910, "U", trans, n, k, dist="wide")
    ra, ca = (n, k) if trans == "N" else (k, n)
    ea = case["lda"] * (ca - 1) + ra
    ec = case["ldc"] * (n - 1) + n
    O = (case["C"][0].copy(), case["C"][1].copy())
    assert oracle.rsyrk("U", trans, n, k, case["alpha"], case["A"], case["lda"], case["beta"], O,
                        case["ldc"]) == 0
    bufs = [tight(case["A"], ea), tight(case["C"], ec)]
    before = [x[0].copy() for x in bufs]
    assert b.mpdd_Rsyrk_host(h, "U", trans, n, k, case["alpha"], bufs[0][1], case["lda"],
                             case["beta"], bufs[1][1], case["ldc"]) == 0
    for (full, _), old, e in zip(bufs, before, (ea, ec)):
        assert np.array_equal(bits(full[e:].ravel()), bits(old[e:].ravel())), trans
    G = planes(bufs[1][1])
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    idx = (i + j * case["ldc"])[i <= j]
    assert ratio(G[0][idx], G[1][idx], O[0][idx], O[1][idx], k) <= RATIO_MAX
    log(f"PARITY host-pointer Rsyrk U {trans} exact-extent arrays ok")


SPLIT_FORMS = {"i8": dict(algo=1), "f64": dict(algo=2), "crt": dict(algo=5)}


@pytest.mark.parametrize("form", sorted(SPLIT_FORMS))
@pytest.mark.parametrize("op", ["NN", "TN", "NT"])
def test_rgemm_host_ex_split_equals_device_call(h, form, op):
    """mpdd_Rgemm_host_ex with a split form: two column chunks, op(A) = A with
    k >= 1024 (the shape that k-slices the first chunk in the plain forms);
    C equals the device mpdd_Rgemm_ex result with the same options bit for
    bit, padding rows included."""
    from paper_2109_13406_amd import binding as b
    from gpu_util import gemm_gpu
    m, n, k = 300, 1100, 1090
    opts = SPLIT_FORMS[form]
    case = W.gemm_case(1950 + len(form), op[0], op[1], m, n, k, dist="wide")
    info, D = gemm_gpu(h, case, opts=opts)
    assert info == 0
    C = pairs(case["C"])
    assert b.mpdd_Rgemm_host_ex(h, opts, op[0], op[1], m, n, k, case["alpha"], pairs(case["A"]),
                                case["lda"], pairs(case["B"]), case["ldb"], case["beta"], C,
                                case["ldc"]) == 0
    G = planes(C)
    assert np.array_equal(bits(G[0]), bits(D[0])) and np.array_equal(bits(G[1]), bits(D[1]))
    log(f"PARITY host-pointer Rgemm_ex {form} {op} {m}x{n}x{k} == device call")


@pytest.mark.parametrize("form", sorted(SPLIT_FORMS))
def test_rsyrk_host_ex_split_equals_device_call(h, form):
    from paper_2109_13406_amd import binding as b
    from gpu_util import syrk_gpu
    n, k = 700, 1030
    opts = SPLIT_FORMS[form]
    case = W.syrk_case(1960 + len(form), "U", "T", n, k, dist="wide")
    info, D = syrk_gpu(h, case, opts=opts)
    assert info == 0
    C = pairs(case["C"])
    assert b.mpdd_Rsyrk_host_ex(h, opts, "U", "T", n, k, case["alpha"], pairs(case["A"]),
                                case["lda"], case["beta"], C, case["ldc"]) == 0
    G = planes(C)
    assert np.array_equal(bits(G[0]), bits(D[0])) and np.array_equal(bits(G[1]), bits(D[1]))


def test_host_ex_plain_and_rejected_options(h):
    """NULL options give mpdd_Rgemm_host's bits; an unknown algo returns
    MPDD_ERR_ARG and an out-of-range moduli count MPDD_ERR_UNSUPPORTED, with
    C unchanged."""
    from paper_2109_13406_amd import binding as b
    m, n, k = 130, 600, 1100
    case = W.gemm_case(1970, "N", "N", m, n, k, dist="wide")
    args = lambda C: ("N", "N", m, n, k, case["alpha"], pairs(case["A"]), case["lda"],
                      pairs(case["B"]), case["ldb"], case["beta"], C, case["ldc"])
    C1, C2 = pairs(case["C"]), pairs(case["C"])
    assert b.mpdd_Rgemm_host(h, *args(C1)) == 0
    assert b.mpdd_Rgemm_host_ex(h, None, *args(C2)) == 0
    assert np.array_equal(bits(C1), bits(C2))
    C0 = pairs(case["C"])
    for bad, code in ((dict(algo=9), b.MPDD_ERR_ARG),
                      (dict(algo=5, nslices=33), b.MPDD_ERR_UNSUPPORTED)):
        C3 = C0.copy()
        assert b.mpdd_Rgemm_host_ex(h, bad, *args(C3)) == code
        assert np.array_equal(bits(C3), bits(C0))
        C3 = C0.copy()
        assert b.mpdd_Rsyrk_host_ex(h, bad, "L", "N", m, k, case["alpha"], pairs(case["A"]),
                                    case["lda"], case["beta"], C3, case["ldc"]) == code
        assert np.array_equal(bits(C3), bits(C0))


@pytest.mark.parametrize("form,op", [("crt", "NT"), ("i8", "NN"), ("crt", "TT")])
def test_rgemm_host_ex_eight_chunks(h, form, op):
    """Eight column chunks (n = 4096 = 8 x 512) through the three chunk
    buffers, the copies back overlapping the next chunk's copies in: C equals
    the device call bit for bit, padding rows included."""
    from paper_2109_13406_amd import binding as b
    from gpu_util import gemm_gpu
    m, n, k = 70, 4096, 300
    opts = SPLIT_FORMS[form]
    case = W.gemm_case(1980 + len(form), op[0], op[1], m, n, k, dist="wide")
    info, D = gemm_gpu(h, case, opts=opts)
    assert info == 0
    C = pairs(case["C"])
    assert b.mpdd_Rgemm_host_ex(h, opts, op[0], op[1], m, n, k, case["alpha"], pairs(case["A"]),
                                case["lda"], pairs(case["B"]), case["ldb"], case["beta"], C,
                                case["ldc"]) == 0
    G = planes(C)
    assert np.array_equal(bits(G[0]), bits(D[0])) and np.array_equal(bits(G[1]), bits(D[1]))
    log(f"PARITY host-pointer Rgemm_ex {form} {op} {m}x{n}x{k}, eight chunks == device call")


@pytest.mark.parametrize("op", ["NN", "TT"])
def test_host_ex_modular_exact_extent(h, op):
    """The modular form through the host-pointer calls on arrays sized exactly
    to their BLAS extent: nothing past any extent is written, and C equals
    the device call bit for bit (Rgemm over two column chunks; Rsyrk)."""
    from paper_2109_13406_amd import binding as b
    from gpu_util import gemm_gpu, syrk_gpu
    opts = SPLIT_FORMS["crt"]
    m, n, k = 300, 1100, 1090
    case = W.gemm_case(1990, op[0], op[1], m, n, k, dist="wide")
    ra, ca = (m, k) if op[0] == "N" else (k, m)
    rb, cb = (k, n) if op[1] == "N" else (n, k)
    ea = case["lda"] * (ca - 1) + ra
    eb = case["ldb"] * (cb - 1) + rb
    ec = case["ldc"] * (n - 1) + m
    info, D = gemm_gpu(h, case, opts=opts)
    assert info == 0
    bufs = [tight(case["A"], ea), tight(case["B"], eb), tight(case["C"], ec)]
    before = [x[0].copy() for x in bufs]
    assert b.mpdd_Rgemm_host_ex(h, opts, op[0], op[1], m, n, k, case["alpha"], bufs[0][1],
                                case["lda"], bufs[1][1], case["ldb"], case["beta"], bufs[2][1],
                                case["ldc"]) == 0
    for (full, _), old, e in zip(bufs, before, (ea, eb, ec)):
        assert np.array_equal(bits(full[e:].ravel()), bits(old[e:].ravel())), op
    G = planes(bufs[2][1])
    assert np.array_equal(bits(G[0]), bits(D[0][:ec])) and np.array_equal(bits(G[1]), bits(D[1][:ec]))
    trans = "N" if op[0] == "N" else "T"
    ns, ks = 260, 300
    case = W.syrk_case(1991, "L", trans, ns, ks, dist="wide")
    ra, ca = (ns, ks) if trans == "N" else (ks, ns)
    ea = case["lda"] * (ca - 1) + ra
    ec = case["ldc"] * (ns - 1) + ns
    info, D = syrk_gpu(h, case, opts=opts)
    assert info == 0
    bufs = [tight(case["A"], ea), tight(case["C"], ec)]
    before = [x[0].copy() for x in bufs]
    assert b.mpdd_Rsyrk_host_ex(h, opts, "L", trans, ns, ks, case["alpha"], bufs[0][1],
                                case["lda"], case["beta"], bufs[1][1], case["ldc"]) == 0
    for (full, _), old, e in zip(bufs, before, (ea, ec)):
        assert np.array_equal(bits(full[e:].ravel()), bits(old[e:].ravel())), trans
    G = planes(bufs[1][1])
    assert np.array_equal(bits(G[0]), bits(D[0][:ec])) and np.array_equal(bits(G[1]), bits(D[1][:ec]))
    log(f"PARITY host-pointer modular Rgemm {op} / Rsyrk L {trans} exact-extent arrays ok")

"""GPU parity of the split (Ozaki) form through the C ABI.

* Slices: scale exponents and every digit bit-identical to the oracle's
  split, padding digits zero (INT8 and FP64 digit widths).
* Products + combine: the split-form Rgemm is bit-identical to the oracle's
  split-form evaluation with the same slice count (the slice products are
  exact integers and the combine runs the same dd steps in the same order).
* Accuracy: with enough slices the result is within 8 k 2^-104 of the plain
  dd oracle, for the uniform and the wide (2^+-20 exponent) input sets; the
  full-size cases search the slice count upward until that holds.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import (compare_full, dev, entries_mask, gemm_gpu, gemm_oracle, log,
                      sampled_gemm_check, sampled_syrk_check, syrk_gpu, syrk_oracle)
from oracle.compare import RATIO_MAX, bits

pytestmark = pytest.mark.gpu

KINDS = {"i8": 1, "f64": 2}


@pytest.fixture(scope="module")
def h():
    import torch
    from paper_2109_13406_amd import binding as b
    handle = b.mpdd_create()
    yield handle
    torch.cuda.synchronize()
    b.mpdd_destroy(handle)


def _widths(kind, k, s):
    """(wfirst, w, qmax) of the library's digits for k terms and s slices."""
    if kind == "i8":
        return oracle.int8_digit_widths(k, s) + (oracle.INT8_QMAX,)
    return oracle.fp64_digit_width(k, s) + (0,)


@pytest.mark.parametrize("kind", ["i8", "f64"])
@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_slices_bit_identical(h, kind, trans, dist):
    import torch
    from paper_2109_13406_amd import binding as b
    algo = KINDS[kind]
    # (3 x 9000 x 16 has nslices*k >= 2^17: 7-bit INT8 digits; 40 x 300 x 20
    # has more 8-bit digits than the slicing kernel keeps in registers)
    for (rows, k, s) in [(70, 90, 16), (1, 1, 3), (130, 200, 9), (3, 9000, 16), (40, 300, 20)]:
        rng = W.streams(11 + rows)[0]
        nr, nc = (rows, k) if trans == "N" else (k, rows)
        ld = W.ld_padded(nr)
        X = W.dd_matrix(rng, nr, nc, ld, dist=dist)
        sr, sl = (1, ld) if trans == "N" else (ld, 1)
        wf, w, qmax = _widths(kind, k, s)
        assert b.mpdd_ozaki_digit_widths(algo, k, s) == (wf, w)
        e_o, q_o = oracle.ozaki_split(rows, k, X, sr, sl, s, wf, w, qmax)
        ldq = 64 * ((k + 63) // 64)
        rows_p = 64 * ((rows + 63) // 64)
        exps = torch.zeros(rows, dtype=torch.int32, device="cuda")
        dt = torch.int8 if kind == "i8" else torch.float64
        q = torch.full((s, rows_p, ldq), 7, dtype=dt, device="cuda")
        info = b.mpdd_ozaki_split(h, algo, trans, rows, k, dev(X), ld, s, exps, q, ldq, rows_p)
        assert info == 0
        torch.cuda.synchronize()
        assert np.array_equal(exps.cpu().numpy(), e_o)
        qg = q.cpu().numpy().astype(np.int64) if kind == "i8" else q.cpu().numpy()
        assert np.array_equal(qg[:, :rows, :k], q_o.astype(qg.dtype)), (kind, trans, rows, k)
        assert not qg[:, rows:, :].any() and not qg[:, :, k:].any()
    log(f"PARITY ozaki slices {kind} {trans} {dist} bit-identical")


def test_int8_slices_carry_chains(h):
    """8-bit INT8 digits that round to 128 are carried into the digit before
    them, through runs of 127: rows built from values whose digits are
    worked out by hand (first digit 20, then 128, or 127 then 128), beside
    0.75 for the scale, give the oracle's carried digits bit for bit."""
    import torch
    from fractions import Fraction
    from paper_2109_13406_amd import binding as b
    vals = [Fraction(20 * 256 + Fraction(511, 4), 256 * 64),
            Fraction(20 * 256 * 256 + 127 * 256 + Fraction(511, 4), 256 * 256 * 64)]
    rows, k, s = 2, 64, 6
    X = (np.zeros(rows * k), np.zeros(rows * k))     # row-major rows: trans "T", ld = k
    for r, x in enumerate(vals):
        X[0][r * k] = 0.75
        for l in range(1, k):
            sign = -1 if l % 2 else 1
            hi = float(x) * sign
            X[0][r * k + l] = hi
            X[1][r * k + l] = float(sign * x - Fraction(hi))
    wf, w, qmax = _widths("i8", k, s)
    assert (wf, w) == (6, 8)
    e_o, q_o = oracle.ozaki_split(rows, k, X, k, 1, s, wf, w, qmax)
    # odd l hold -x (no carry: -128 fits), even l > 0 hold x (carried)
    assert [int(v) for v in q_o[:, 0, 2]] == [21, -128, -64, 0, 0, 0]
    assert [int(v) for v in q_o[:, 1, 2]] == [21, -128, -128, -64, 0, 0]
    assert [int(v) for v in q_o[:, 0, 1]] == [-20, -128, 64, 0, 0, 0]
    exps = torch.zeros(rows, dtype=torch.int32, device="cuda")
    q = torch.full((s, 64, 64), 7, dtype=torch.int8, device="cuda")
    info = b.mpdd_ozaki_split(h, b.MPDD_OZAKI_I8, "T", rows, k, dev(X), k, s, exps, q, 64, 64)
    assert info == 0
    torch.cuda.synchronize()
    assert np.array_equal(exps.cpu().numpy(), e_o)
    qg = q.cpu().numpy().astype(np.int64)
    assert np.array_equal(qg[:, :rows, :k], q_o.astype(np.int64))
    log("PARITY ozaki int8 carry chains bit-identical")


SHAPES = [(1, 1, 1), (70, 90, 33), (129, 130, 200), (200, 64, 65), (300, 270, 130)]
VARIANTS = (0, 1, 2, 3, 4, 5, 6, 7, 8)   # INT8 product tilings (see the tile_id options)


@pytest.mark.parametrize("kind", ["i8", "f64"])
@pytest.mark.parametrize("op", W.OPS)
def test_split_gemm_bit_identical_to_split_oracle(h, kind, op):
    algo = KINDS[kind]
    for (m, n, k) in SHAPES:
        for dist in ("uniform", "wide"):
            s = 9 if kind == "i8" else 4
            case = W.gemm_case(60 + m + k, op[0], op[1], m, n, k, dist=dist)
            wf, w, qmax = _widths(kind, k, s)
            O = (case["C"][0].copy(), case["C"][1].copy())
            assert oracle.ozaki_rgemm(op[0], op[1], m, n, k, case["alpha"], case["A"], case["lda"],
                                      case["B"], case["ldb"], case["beta"], O, case["ldc"], s, wf,
                                      w, qmax) == 0
            # every INT8 product variant (workgroup tiling) must give the same bits
            for var in (VARIANTS if kind == "i8" else (-1,)):
                info, G = gemm_gpu(h, case, opts=dict(algo=algo, nslices=s, tile_id=var))
                assert info == 0
                assert np.array_equal(bits(G[0]), bits(O[0])), (kind, op, m, n, k, dist, var)
                assert np.array_equal(bits(G[1]), bits(O[1])), (kind, op, m, n, k, dist, var)
    log(f"PARITY ozaki {kind} {op} bit-identical to the split oracle")


@pytest.mark.parametrize("kind", ["i8", "f64"])
@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_split_gemm_reaches_dd_accuracy(h, kind, dist):
    algo = KINDS[kind]
    m, n, k = 150, 140, 300
    case = W.gemm_case(70, "N", "T", m, n, k, dist=dist)
    O = gemm_oracle(case)
    s = {("i8", "uniform"): 16, ("i8", "wide"): 22, ("f64", "uniform"): 7,
         ("f64", "wide"): 9}[(kind, dist)]
    info, G = gemm_gpu(h, case, opts=dict(algo=algo, nslices=s))
    assert info == 0
    r = compare_full(f"ozaki {kind} {dist} s={s} NT {m}x{n}x{k}", G, O, m, n, k, case["ldc"],
                     C0=case["C"], case=case)
    assert r <= RATIO_MAX


def test_split_semantics(h):
    """beta = 0 with NaN C, alpha = 0, and an unsupported slice count."""
    from paper_2109_13406_amd import binding as b
    case = W.gemm_case(71, "T", "N", 40, 30, 50, beta_zero=True, c_nan=True)
    O = gemm_oracle(case)
    info, G = gemm_gpu(h, case, opts=dict(algo=b.MPDD_OZAKI_I8, nslices=16))
    assert info == 0
    assert compare_full("ozaki beta0", G, O, 40, 30, 50, case["ldc"], C0=case["C"],
                        case=case) <= RATIO_MAX
    case = W.gemm_case(72, "N", "N", 20, 20, 20)
    case["alpha"] = (0.0, 0.0)
    O = gemm_oracle(case)
    info, G = gemm_gpu(h, case, opts=dict(algo=b.MPDD_OZAKI_F64))
    assert info == 0
    assert np.array_equal(bits(G[0]), bits(O[0]))
    info, _ = gemm_gpu(h, W.gemm_case(73, "N", "N", 8, 8, 8),
                       opts=dict(algo=b.MPDD_OZAKI_I8, nslices=41))
    assert info == b.MPDD_ERR_UNSUPPORTED
    info, _ = gemm_gpu(h, W.gemm_case(74, "N", "N", 8, 8, 8),
                       opts=dict(algo=b.MPDD_OZAKI_I8, nslices=12, tile_id=9))
    assert info == b.MPDD_ERR_UNSUPPORTED


SYRK_SHAPES = [(1, 1), (70, 33), (130, 200), (300, 130)]
SYRK_VARIANTS = (0, 2, 3, 4, 5, 6, 7, 8)   # INT8 tilings with square tiles


def _split_syrk_reference(case, kind, s):
    """The split oracle's Rgemm of op(A) and op(A)^T (the whole square; only
    the case's triangle is compared)."""
    n, k, trans = case["n"], case["k"], case["trans"].upper()
    wf, w, qmax = _widths(kind, k, s)
    O = (case["C"][0].copy(), case["C"][1].copy())
    assert oracle.ozaki_rgemm(trans, "T" if trans == "N" else "N", n, n, k, case["alpha"],
                              case["A"], case["lda"], case["A"], case["lda"], case["beta"], O,
                              case["ldc"], s, wf, w, qmax) == 0
    return O


def _check_split_syrk(G, O, case, what):
    """Triangle bit-identical to O; every other stored word (the opposite
    triangle's NaN sentinel, the padding rows) bit-identical to the input."""
    idx = entries_mask(case["n"], case["n"], case["ldc"], case["uplo"].upper())
    rest = np.ones(G[0].shape[0], bool)
    rest[idx] = False
    for p in (0, 1):
        assert np.array_equal(bits(G[p])[idx], bits(O[p])[idx]), what
        assert np.array_equal(bits(G[p])[rest], bits(case["C"][p])[rest]), what


@pytest.mark.parametrize("kind", ["i8", "f64"])
@pytest.mark.parametrize("uplo", ["U", "L"])
@pytest.mark.parametrize("trans", ["N", "T"])
def test_split_syrk_bit_identical_to_split_oracle(h, kind, uplo, trans):
    """Split-form Rsyrk: op(B) = op(A)^T takes op(A)'s slices, only the
    triangle's tiles are multiplied and only the triangle is combined; the
    triangle equals the split oracle's Rgemm of op(A) and op(A)^T bit for bit
    for every square INT8 tiling, and nothing else of C changes."""
    algo = KINDS[kind]
    s = 9 if kind == "i8" else 4
    for (n, k) in SYRK_SHAPES:
        for dist in ("uniform", "wide"):
            case = W.syrk_case(80 + n + k, uplo, trans, n, k, dist=dist)
            O = _split_syrk_reference(case, kind, s)
            for var in (SYRK_VARIANTS if kind == "i8" else (-1,)):
                info, G = syrk_gpu(h, case, opts=dict(algo=algo, nslices=s, tile_id=var))
                assert info == 0
                _check_split_syrk(G, O, case, (kind, uplo, trans, n, k, dist, var))
    log(f"PARITY ozaki syrk {kind} {uplo}{trans} bit-identical to the split oracle")


@pytest.mark.parametrize("kind,n", [("i8", 2048), ("f64", 1024)])
@pytest.mark.parametrize("uplo", ["U", "L"])
def test_split_syrk_blocked_triangle_walk(h, kind, n, uplo):
    """With a multiple of 8 tiles per side the triangle's tiles are walked in
    8 x 8 blocks (off-diagonal blocks, then diagonal ones) dealt to the XCDs
    in equal runs: every tile of the triangle is computed once, bit for bit
    as the split oracle; beta = 0 never reads C (all NaN)."""
    algo = KINDS[kind]
    s, k = 6, 64
    for trans, beta_zero in (("N", False), ("T", True)):
        case = W.syrk_case(90 + n, uplo, trans, n, k, beta_zero=beta_zero)
        O = _split_syrk_reference(case, kind, s)
        info, G = syrk_gpu(h, case, opts=dict(algo=algo, nslices=s))
        assert info == 0
        _check_split_syrk(G, O, case, (kind, n, uplo, trans, beta_zero))
    log(f"PARITY ozaki syrk {kind} n={n} {uplo} blocked triangle walk bit-identical")


def test_split_syrk_semantics(h):
    """alpha = 0 scales the triangle only (bit-identical to the oracle's
    Rsyrk); the 256 x 128 INT8 tiling is rejected for a triangle, nothing
    enqueued."""
    from paper_2109_13406_amd import binding as b
    case = W.syrk_case(91, "U", "T", 60, 40)
    case["alpha"] = (0.0, 0.0)
    O = syrk_oracle(case)
    for algo in (b.MPDD_OZAKI_I8, b.MPDD_OZAKI_F64):
        info, G = syrk_gpu(h, case, opts=dict(algo=algo, nslices=8))
        assert info == 0
        for p in (0, 1):
            assert np.array_equal(bits(G[p]), bits(O[p]))
    case = W.syrk_case(92, "L", "N", 60, 40)
    info, G = syrk_gpu(h, case, opts=dict(algo=b.MPDD_OZAKI_I8, nslices=8, tile_id=1))
    assert info == b.MPDD_ERR_UNSUPPORTED
    for p in (0, 1):
        assert np.array_equal(bits(G[p]), bits(case["C"][p]))


@pytest.mark.parametrize("uplo,trans", [("U", "N"), ("L", "N"), ("U", "T"), ("L", "T")])
def test_split_syrk_config2_size(h, uplo, trans):
    """Config-2 shape n = k = 8192 in the INT8 split form with the slice count
    the benchmark times (12): within 8 k 2^-104 of the plain dd oracle on
    sampled entries of the triangle."""
    import torch
    from paper_2109_13406_amd import binding as b
    n = k = 8192
    case = W.syrk_case_device(W.BASE_SEED + 2, uplo, trans, n, k)
    r = sampled_syrk_check(h, f"config2 ozaki syrk i8 {uplo}{trans} n={n} k={k} s=12", case,
                           opts=dict(algo=b.MPDD_OZAKI_I8, nslices=12), count=W.CONFIG3_SAMPLE,
                           seed=W.BASE_SEED + 2)
    del case
    torch.cuda.empty_cache()
    assert r <= RATIO_MAX


def _digit_value(digits, wf, w):
    """(hi, lo) of the dd value whose digits, as the slicing rounds them, are
    `digits` (first digit wf bits wide, later ones w bits)."""
    from fractions import Fraction
    x = sum(Fraction(d, 2 ** (wf + w * t)) for t, d in enumerate(digits))
    hi = float(x)
    return hi, float(x - Fraction(hi))


@pytest.mark.parametrize("k,digit", [(10922, 127), (43690, 63)], ids=["w8-k10922", "w7-k43690"])
def test_int8_accumulators_at_the_exactness_limit(h, k, digit):
    """Largest k of each INT8 digit width for 12 slices (12 k just below
    2^17, then just below 2^19), with inputs whose digits are all at their
    largest (first digit 63, later ones `digit`): every anti-diagonal sum of
    the last diagonal reaches 90-97 % of 2^31.  The int32 accumulation on the
    matrix cores must equal the oracle's int64 evaluation bit for bit, for
    every product tiling, with all products positive and with all negative;
    one more k for the 7-bit form is rejected."""
    import torch
    from paper_2109_13406_amd import binding as b
    s, m, n = 12, 16, 16
    wf, w, qmax = _widths("i8", k, s)
    assert (wf, w) == ((6, 8) if digit == 127 else (6, 7))
    hi, lo = _digit_value([63] + [digit] * (s - 1), wf, w)
    # the largest last-diagonal sum: sum over t + u = 13 of q_t q_u, k times
    top = (2 * 63 * digit + (s - 2) * digit * digit) * k
    assert 0.9 * 2 ** 31 < top < 2 ** 31
    for sign_a in (1.0, -1.0):
        A = (np.full(m * k, sign_a * hi), np.full(m * k, sign_a * lo))
        B = (np.full(k * n, hi), np.full(k * n, lo))
        C = (np.zeros(m * n), np.zeros(m * n))
        # the oracle's digits are the intended ones
        _, q = oracle.ozaki_split(1, k, A, 0, 1, s, wf, w, qmax)
        assert [int(v) for v in q[:, 0, 0]] == [int(sign_a) * v for v in [63] + [digit] * (s - 1)]
        O = (C[0].copy(), C[1].copy())
        assert oracle.ozaki_rgemm("N", "N", m, n, k, (1.0, 0.0), A, m, B, k, (0.0, 0.0), O, m,
                                  s, wf, w, qmax) == 0
        print(f"int8 limit k={k} digit={digit} sign={sign_a}", flush=True)
        for var in VARIANTS:
            Cd = dev(C)
            info = b.mpdd_Rgemm_ex(h, dict(algo=b.MPDD_OZAKI_I8, nslices=s, tile_id=var), "N",
                                   "N", m, n, k, (1.0, 0.0), dev(A), m, dev(B), k, (0.0, 0.0),
                                   Cd, m)
            assert info == 0
            G = tuple(x.cpu().numpy() for x in Cd)
            assert np.array_equal(bits(G[0]), bits(O[0])), (k, sign_a, var)
            assert np.array_equal(bits(G[1]), bits(O[1])), (k, sign_a, var)
    if w == 7:
        # s * (k + 1) = 2^19: no exact width, nothing enqueued
        with pytest.raises(ValueError):
            b.mpdd_ozaki_digit_widths(b.MPDD_OZAKI_I8, k + 1, s)
        z = lambda cnt: tuple(torch.zeros(cnt, dtype=torch.float64, device="cuda")
                              for _ in range(2))
        Cz = z(m * n)
        info = b.mpdd_Rgemm_ex(h, dict(algo=b.MPDD_OZAKI_I8, nslices=s), "N", "N", m, n, k + 1,
                               (1.0, 0.0), z(m * (k + 1)), m, z((k + 1) * n), k + 1, (0.0, 0.0),
                               Cz, m)
        assert info == b.MPDD_ERR_UNSUPPORTED
        torch.cuda.synchronize()
        assert not Cz[0].any() and not Cz[1].any()
    log(f"PARITY ozaki int8 at the exactness limit k={k} (w={w}) bit-identical, all variants")


def slice_search(h, kind, n, dist, start, stop):
    """Smallest slice count whose sampled ratio vs the dd oracle is <= 8, on
    the benchmark's config-3 inputs and entries (so the slice count the
    benchmark times is the one this search finds and checks)."""
    import torch
    algo = KINDS[kind]
    case = W.gemm_case_device(W.BASE_SEED + 3, "N", "N", n, n, n, dist=dist)
    C0 = tuple(x.clone() for x in case["C"])
    for s in range(start, stop + 1):
        for dst, src in zip(case["C"], C0):
            dst.copy_(src)
        r = sampled_gemm_check(h, f"config3 ozaki {kind} n={n} {dist} s={s}", case,
                               opts=dict(algo=algo, nslices=s), count=W.CONFIG3_SAMPLE,
                               seed=W.BASE_SEED + 3)
        if r <= RATIO_MAX:
            del case, C0
            torch.cuda.empty_cache()
            return s, r
    return None, None


@pytest.mark.parametrize("n", [2048, 8192])
@pytest.mark.parametrize("kind", ["i8", "f64"])
@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_config3_slice_count_search(h, n, kind, dist):
    """Config 3: the slice count is searched upward from below any count
    that can reach dd accuracy (INT8 from 8 slices, FP64 from 3) until the
    result is within 8 k 2^-104 of the oracle; the counts below it are
    checked and fail, the one found passes."""
    start, stop = {"i8": (8, 24), "f64": (3, 10)}[kind]
    s, r = slice_search(h, kind, n, dist, start, stop)
    log(f"CONFIG3 {kind} n={n} {dist}: slices={s} ratio={r}")
    assert s is not None and s > start

"""GPU parity of the modular (Chinese-remainder) split form through the C ABI.

* Residues: scale exponents and every int8 residue bit-identical to the
  modular oracle (oracle/crt.py), padding zero.
* Rgemm / Rsyrk: within 2^-100 (|C| + 2|beta C0|) of the oracle's exactly
  rounded result (the per-modulus products are exact integers and the
  reconstruction is exact; only the final conversion and the alpha / beta
  update round), for every op form, both input sets, ragged shapes over
  several 256 x 256 tiles; every product tiling gives the same bits.
* int32 headroom: k = 2^17 - 1 with the modulus-256 residues all -128.
* Accuracy: within 8 k 2^-104 of the plain dd oracle; at the benchmark's
  8192^3 inputs the moduli count is searched upward until that holds.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from gpu_util import (compare_full, dev, entries_mask, gemm_gpu, gemm_oracle, log,
                      sampled_gemm_check, syrk_gpu)
from oracle import crt as CRT
from oracle.compare import RATIO_MAX, bits

pytestmark = pytest.mark.gpu

TILINGS = (5, 6, 8)     # the INT8 product tilings (tile_id) the modular form runs on
TOL = 2.0 ** -100


@pytest.fixture(scope="module")
def h():
    import torch
    from paper_2109_13406_amd import binding as b
    handle = b.mpdd_create()
    yield handle
    torch.cuda.synchronize()
    b.mpdd_destroy(handle)


def _algo():
    from paper_2109_13406_amd import binding as b
    return b.MPDD_OZAKI_CRT


def _check_close(G, R, C0, beta, idx, what):
    """|G - R| <= 2^-100 (|R| + 2 |beta| |C0|) on the flat entries idx."""
    gh, gl, rh, rl = G[0][idx], G[1][idx], R[0][idx], R[1][idx]
    diff = np.abs((gh - rh) + (gl - rl))
    tol = TOL * (np.abs(rh) + 2.0 * abs(beta[0]) * np.abs(C0[0][idx]))
    bad = ~(diff <= tol)
    assert not bad.any(), (what, int(bad.sum()), float(np.max(diff / np.maximum(tol, 1e-300))))


@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_crt_residues_bit_identical(h, trans, dist):
    import torch
    from paper_2109_13406_amd import binding as b
    for (rows, k, count) in [(1, 1, 1), (70, 90, 27), (200, 330, 12), (130, 200, 32),
                             (3, 9000, 27)]:
        rng = W.streams(31 + rows)[0]
        nr, nc = (rows, k) if trans == "N" else (k, rows)
        ld = W.ld_padded(nr)
        X = W.dd_matrix(rng, nr, nc, ld, dist=dist)
        if rows > 3:                        # a zero row of the row operand
            for p in (0, 1):
                if trans == "N":
                    X[p][2 + np.arange(k) * ld] = 0.0
                else:
                    X[p][np.arange(k) + 2 * ld] = 0.0
        p_bits = CRT.exponent(k, count)
        assert b.mpdd_ozaki_crt_exponent(k, count) == p_bits
        hi, lo = CRT.row_operand(trans, rows, k, X, ld)
        e_o = CRT.scale_exponents(hi)
        q_o = CRT.residues(CRT.integers(hi, lo, e_o, p_bits), count)
        ldq = 64 * ((k + 63) // 64)
        rows_p = 64 * ((rows + 63) // 64)
        exps = torch.zeros(rows, dtype=torch.int32, device="cuda")
        q = torch.full((count, rows_p, ldq), 7, dtype=torch.int8, device="cuda")
        print(f"crt residues {trans} {dist} rows={rows} k={k} count={count}", flush=True)
        info = b.mpdd_ozaki_split(h, _algo(), trans, rows, k, dev(X), ld, count, exps, q, ldq,
                                  rows_p)
        assert info == 0
        torch.cuda.synchronize()
        assert np.array_equal(exps.cpu().numpy(), e_o)
        qg = q.cpu().numpy().astype(np.int64)
        assert np.array_equal(qg[:, :rows, :k], q_o), (trans, dist, rows, k, count)
        assert not qg[:, rows:, :].any() and not qg[:, :, k:].any()
    log(f"PARITY crt residues {trans} {dist} bit-identical")


def _crt_reference(case, count):
    O = (case["C"][0].copy(), case["C"][1].copy())
    CRT.crt_rgemm(case["transa"], case["transb"], case["m"], case["n"], case["k"],
                  case["alpha"], case["A"], case["lda"], case["B"], case["ldb"], case["beta"], O,
                  case["ldc"], count)
    return O


GEMM_SHAPES = [(1, 1, 1, 27), (70, 90, 33, 27), (300, 270, 130, 27), (260, 520, 64, 12)]


@pytest.mark.parametrize("op", W.OPS)
def test_crt_gemm_matches_crt_oracle(h, op):
    for (m, n, k, count) in GEMM_SHAPES:
        for dist in ("uniform", "wide"):
            if dist == "wide" and m * n > 100000:
                continue
            case = W.gemm_case(160 + m + k, op[0], op[1], m, n, k, dist=dist)
            print(f"crt gemm {op} {m}x{n}x{k} {dist} count={count}", flush=True)
            R = _crt_reference(case, count)
            idx = entries_mask(m, n, case["ldc"])
            first = None
            for var in TILINGS:
                info, G = gemm_gpu(h, case, opts=dict(algo=_algo(), nslices=count, tile_id=var))
                assert info == 0
                if first is None:
                    _check_close(G, R, case["C"], case["beta"], idx, (op, m, n, k, dist))
                    # entries outside the m x n block are untouched
                    rest = np.ones(G[0].shape[0], bool)
                    rest[idx] = False
                    for p in (0, 1):
                        assert np.array_equal(bits(G[p])[rest], bits(case["C"][p])[rest])
                    first = G
                else:
                    for p in (0, 1):
                        assert np.array_equal(bits(G[p]), bits(first[p])), (op, m, n, k, var)
    log(f"PARITY crt gemm {op} within 2^-100 of the modular oracle, all tilings identical")


@pytest.mark.parametrize("uplo", ["U", "L"])
@pytest.mark.parametrize("trans", ["N", "T"])
def test_crt_syrk_matches_crt_oracle(h, uplo, trans):
    """op(B) = op(A)^T reuses op(A)'s residues, only the triangle's tiles are
    multiplied and reconstructed; the rest of C keeps its bits."""
    count = 27
    for (n, k) in [(1, 1), (130, 200), (300, 70)]:
        for dist in ("uniform", "wide"):
            case = W.syrk_case(180 + n + k, uplo, trans, n, k, dist=dist)
            tr = trans.upper()
            # the whole square (the opposite triangle's NaN sentinel read as 0)
            R = tuple(np.nan_to_num(x, nan=0.0) for x in case["C"])
            CRT.crt_rgemm(tr, "T" if tr == "N" else "N", n, n, k, case["alpha"], case["A"],
                          case["lda"], case["A"], case["lda"], case["beta"], R, case["ldc"],
                          count)
            idx = entries_mask(n, n, case["ldc"], uplo)
            rest = np.ones(case["C"][0].shape[0], bool)
            rest[idx] = False
            first = None
            print(f"crt syrk {uplo}{trans} n={n} k={k} {dist}", flush=True)
            for var in TILINGS:
                info, G = syrk_gpu(h, case, opts=dict(algo=_algo(), nslices=count, tile_id=var))
                assert info == 0
                if first is None:
                    _check_close(G, R, case["C"], case["beta"], idx, (uplo, trans, n, k, dist))
                    for p in (0, 1):
                        assert np.array_equal(bits(G[p])[rest], bits(case["C"][p])[rest])
                    first = G
                else:
                    for p in (0, 1):
                        assert np.array_equal(bits(G[p]), bits(first[p])), (uplo, trans, n, var)
    log(f"PARITY crt syrk {uplo}{trans} within 2^-100 of the modular oracle")


def test_crt_int32_headroom(h):
    """k = 2^17 - 1 (the largest k the form takes) with every entry of A and
    B equal to 1/2 - 2^(7-P): the integers are 2^(P-1) - 128, so every
    modulus-256 residue is -128 and that plane's sums reach k 2^14 =
    2^31 - 2^14.  The result is k (1/2 - 2^(7-P))^2 within 2^-100; k = 2^17
    is rejected with nothing enqueued."""
    import torch
    from paper_2109_13406_amd import binding as b
    k, m, n, count = (1 << 17) - 1, 16, 16, 32
    p = CRT.exponent(k, count)
    assert b.mpdd_ozaki_crt_exponent(k, count) == p
    v = Fraction(1, 2) - Fraction(2) ** (7 - p)
    hi = float(v)
    lo = float(v - Fraction(hi))
    ints = CRT.integers(np.array([[hi]]), np.array([[lo]]), CRT.scale_exponents(np.array([[hi]])),
                        p)
    assert ints[0, 0] == 2 ** (p - 1) - 128
    assert CRT.residues(ints, 1)[0, 0, 0] == -128
    z = lambda cnt, val: tuple(torch.full((cnt,), x, dtype=torch.float64, device="cuda")
                               for x in val)
    Cd = z(m * n, (0.0, 0.0))
    info = b.mpdd_Rgemm_ex(h, dict(algo=_algo(), nslices=count), "N", "N", m, n, k, (1.0, 0.0),
                           z(m * k, (hi, lo)), m, z(k * n, (hi, lo)), k, (0.0, 0.0), Cd, m)
    assert info == 0
    torch.cuda.synchronize()
    G = tuple(x.cpu().numpy() for x in Cd)
    want = k * v * v
    rh = float(want)
    R = (np.full(m * n, rh), np.full(m * n, float(want - Fraction(rh))))
    _check_close(G, R, R, (0.0, 0.0), np.arange(m * n), "headroom")
    Cz = z(m * n, (0.0, 0.0))
    info = b.mpdd_Rgemm_ex(h, dict(algo=_algo(), nslices=count), "N", "N", m, n, k + 1,
                           (1.0, 0.0), z(m * (k + 1), (hi, lo)), m, z((k + 1) * n, (hi, lo)),
                           k + 1, (0.0, 0.0), Cz, m)
    assert info == b.MPDD_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert not Cz[0].any() and not Cz[1].any()
    log(f"PARITY crt int32 headroom k={k} within 2^-100, k={k + 1} rejected")


def test_crt_semantics(h):
    """beta = 0 with NaN C, alpha = 0 (bit-identical to the oracle's Rgemm),
    too many moduli, too few for k, a tiling the form does not run on, the
    no-allocation entry."""
    from paper_2109_13406_amd import binding as b
    case = W.gemm_case(191, "T", "N", 40, 30, 50, beta_zero=True, c_nan=True)
    R = _crt_reference(case, 20)
    info, G = gemm_gpu(h, case, opts=dict(algo=_algo(), nslices=20))
    assert info == 0
    _check_close(G, R, (np.zeros_like(R[0]),) * 2, (0.0, 0.0),
                 entries_mask(40, 30, case["ldc"]), "beta0")
    case = W.gemm_case(192, "N", "N", 20, 20, 20)
    case["alpha"] = (0.0, 0.0)
    O = gemm_oracle(case)
    info, G = gemm_gpu(h, case, opts=dict(algo=_algo()))
    assert info == 0
    assert np.array_equal(bits(G[0]), bits(O[0])) and np.array_equal(bits(G[1]), bits(O[1]))
    for count in (33, 2):
        case = W.gemm_case(193, "N", "N", 8, 8, 8192)
        info, G = gemm_gpu(h, case, opts=dict(algo=_algo(), nslices=count))
        assert info == b.MPDD_ERR_UNSUPPORTED, count
        assert np.array_equal(bits(G[0]), bits(case["C"][0]))
    for var in (0, 7, 9):
        info, _ = gemm_gpu(h, W.gemm_case(194, "N", "N", 8, 8, 8),
                           opts=dict(algo=_algo(), nslices=12, tile_id=var))
        assert info == b.MPDD_ERR_UNSUPPORTED, var
    case = W.gemm_case(195, "N", "N", 8, 8, 8)
    A, B, C = dev(case["A"]), dev(case["B"]), dev(case["C"])
    info = b.mpdd_Rgemm_noalloc(h, dict(algo=_algo()), "N", "N", 8, 8, 8, case["alpha"], A, 8,
                                B, 8, case["beta"], C, 8)
    assert info == b.MPDD_ERR_UNSUPPORTED


@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_crt_reaches_dd_accuracy(h, dist):
    m, n, k = 150, 140, 300
    case = W.gemm_case(170, "N", "T", m, n, k, dist=dist)
    O = gemm_oracle(case)
    count = {"uniform": 26, "wide": 28}[dist]
    info, G = gemm_gpu(h, case, opts=dict(algo=_algo(), nslices=count))
    assert info == 0
    r = compare_full(f"crt {dist} moduli={count} NT {m}x{n}x{k}", G, O, m, n, k, case["ldc"],
                     C0=case["C"], case=case)
    assert r <= RATIO_MAX


def crt_search(h, n, dist, start, stop):
    """Smallest moduli count whose sampled ratio vs the dd oracle is <= 8, on
    the benchmark's inputs and entries."""
    import torch
    case = W.gemm_case_device(W.BASE_SEED + 3, "N", "N", n, n, n, dist=dist)
    C0 = tuple(x.clone() for x in case["C"])
    for count in range(start, stop + 1):
        for dst, src in zip(case["C"], C0):
            dst.copy_(src)
        r = sampled_gemm_check(h, f"crt n={n} {dist} moduli={count}", case,
                               opts=dict(algo=_algo(), nslices=count), count=W.CONFIG3_SAMPLE,
                               seed=W.BASE_SEED + 3)
        if r <= RATIO_MAX:
            del case, C0
            torch.cuda.empty_cache()
            return count, r
    return None, None


@pytest.mark.parametrize("n", [2048, 8192])
@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_crt_moduli_count_search(h, n, dist):
    """The moduli count is searched upward from a count too small for dd
    accuracy until the sampled result is within 8 k 2^-104 of the oracle."""
    count, r = crt_search(h, n, dist, 22, 32)
    log(f"CRT n={n} {dist}: moduli={count} ratio={r}")
    assert count is not None and count > 22


def _check_close_c(G, R, RP, C0, alpha, beta, idx, what):
    """Complex entries: each part within 2^-99 ((|alpha_r| + |alpha_i|) |P|_1
    + (|beta_r| + |beta_i|) |C0|_1) of the oracle's, |.|_1 = |re| + |im|, P the
    oracle's alpha = 1, beta = 0 product."""
    pmag = np.abs(RP[0][idx]) + np.abs(RP[2][idx])
    cmag = np.abs(C0[0][idx]) + np.abs(C0[2][idx])
    tol = 2.0 ** -99 * ((abs(alpha[0][0]) + abs(alpha[1][0])) * pmag
                        + (abs(beta[0][0]) + abs(beta[1][0])) * cmag)
    for part in (0, 2):
        diff = np.abs((G[part][idx] - R[part][idx]) + (G[part + 1][idx] - R[part + 1][idx]))
        bad = ~(diff <= tol)
        assert not bad.any(), (what, part, int(bad.sum()))


@pytest.mark.parametrize("op", W.COPS, ids=[a + b for a, b in W.COPS])
def test_crt_cgemm_matches_crt_oracle(h, op):
    """Complex modular form (three residue products per modulus): every op
    form, ragged shapes over several tiles, within the dd rounding of the
    final steps of the exactly rounded complex modular oracle; the 256 x 256
    tilings give the same bits."""
    from paper_2109_13406_amd import binding as b
    count = 26
    for (m, n, k, dist) in [(1, 1, 1, "uniform"), (70, 90, 33, "wide"),
                            (260, 270, 64, "uniform")]:
        c = W.cgemm_case(4100 + m + k, op[0], op[1], m, n, k, dist=dist)
        print(f"crt cgemm {op} {m}x{n}x{k} {dist}", flush=True)
        R = tuple(x.copy() for x in c["C"])
        CRT.crt_cgemm(op[0], op[1], m, n, k, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"],
                      c["beta"], R, c["ldc"], count)
        RP = tuple(np.zeros_like(x) for x in c["C"])
        CRT.crt_cgemm(op[0], op[1], m, n, k, ((1.0, 0.0), (0.0, 0.0)), c["A"], c["lda"], c["B"],
                      c["ldb"], ((0.0, 0.0), (0.0, 0.0)), RP, c["ldc"], count)
        idx = entries_mask(m, n, c["ldc"])
        first = None
        for var in TILINGS:
            A, B, C = (tuple(dev((x,))[0] for x in c[key]) for key in ("A", "B", "C"))
            info = b.mpdd_Cgemm_ex(h, dict(algo=_algo(), nslices=count, tile_id=var), op[0],
                                   op[1], m, n, k, c["alpha"], A, c["lda"], B, c["ldb"],
                                   c["beta"], C, c["ldc"])
            assert info == 0
            G = tuple(x.cpu().numpy() for x in C)
            if first is None:
                _check_close_c(G, R, RP, c["C"], c["alpha"], c["beta"], idx, (op, m, n, k))
                first = G
            else:
                for p in range(4):
                    assert np.array_equal(bits(G[p]), bits(first[p])), (op, m, n, k, var)
    log(f"PARITY crt cgemm {op} within 2^-99 of the complex modular oracle")


@pytest.mark.parametrize("uplo,trans", [("U", "N"), ("L", "N"), ("U", "T"), ("L", "T")])
def test_crt_syrk_config2_size(h, uplo, trans):
    """Rsyrk n = k = 8192 (the headline Rsyrk shape) in the modular form with
    the moduli count the benchmark finds (25): within 8 k 2^-104 of the dd
    oracle on sampled entries of the triangle."""
    import torch
    from gpu_util import sampled_syrk_check
    n = k = 8192
    case = W.syrk_case_device(W.BASE_SEED + 2, uplo, trans, n, k)
    r = sampled_syrk_check(h, f"crt syrk {uplo}{trans} n={n} k={k} moduli=25", case,
                           opts=dict(algo=_algo(), nslices=25), count=W.CONFIG3_SAMPLE,
                           seed=W.BASE_SEED + 2)
    del case
    torch.cuda.empty_cache()
    assert r <= RATIO_MAX


@pytest.mark.parametrize("op", ["TN", "NT", "TT"])
def test_crt_gemm_8192_op_forms(h, op):
    """The other op forms at 8192^3 with the benchmark's 25 moduli, sampled
    against the dd oracle."""
    import torch
    n = 8192
    case = W.gemm_case_device(W.BASE_SEED + 3, op[0], op[1], n, n, n)
    r = sampled_gemm_check(h, f"crt {op} n={n} moduli=25", case,
                           opts=dict(algo=_algo(), nslices=25), count=W.CONFIG3_SAMPLE,
                           seed=W.BASE_SEED + 3)
    del case
    torch.cuda.empty_cache()
    assert r <= RATIO_MAX

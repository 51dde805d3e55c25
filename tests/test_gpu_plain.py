"""GPU parity of the plain dd Rgemm / Rsyrk (through the C ABI) against the
CPU oracle, on small seeded cases that span several tiles with ragged tails,
plus the BLAS semantics (beta = 0, alpha = 0, k = 0, quick returns, padding,
opposite triangle) and the worked example."""
import numpy as np
import pytest

import oracle
import pins
import workloads as W
from gpu_util import (compare_full, dev, gemm_gpu, gemm_oracle, host, log, syrk_gpu,
                      syrk_oracle)
from oracle.compare import RATIO_MAX, bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available()
    from paper_2109_13406_amd import binding as b
    handle = b.mpdd_create()
    yield handle
    torch.cuda.synchronize()
    b.mpdd_destroy(handle)


def test_worked_example_bit_exact(h):
    from paper_2109_13406_amd import binding as b
    alpha, beta, v = pins.read_worked_example()
    z = np.zeros(9)
    for ta in "NT":
        for tb in "NT":
            A = v["A"] if ta == "N" else v["A"].T
            B = v["B"] if tb == "N" else v["B"].T
            for algo in (b.MPDD_PLAIN, b.MPDD_PLAIN_ACCURATE):
                case = dict(transa=ta, transb=tb, m=3, n=3, k=3, alpha=(alpha, 0.0),
                            beta=(beta, 0.0), A=(pins.colmajor(A), z.copy()), lda=3,
                            B=(pins.colmajor(B), z.copy()), ldb=3,
                            C=(pins.colmajor(v["C"]), z.copy()), ldc=3)
                info, G = gemm_gpu(h, case, opts=dict(algo=algo))
                assert info == 0
                assert np.array_equal(G[0], pins.colmajor(v["ANSWER"])), (ta, tb, algo, G[0])
                assert np.all(G[1] == 0.0)


def test_config0_rgemm_256(h):
    """Config 0: NN, m = n = k = 256, ld 256."""
    case = W.gemm_case(W.BASE_SEED + 0, "N", "N", 256, 256, 256, padded=False)
    O = gemm_oracle(case)
    info, G = gemm_gpu(h, case)
    assert info == 0
    r = compare_full("config0 NN 256 plain", G, O, 256, 256, 256, 256, case=case)
    assert r <= RATIO_MAX


SHAPES = [(1, 1, 1), (97, 131, 77), (65, 1, 300), (1, 200, 5), (130, 70, 33), (64, 64, 64),
          (200, 190, 1)]


@pytest.mark.parametrize("op", W.OPS)
@pytest.mark.parametrize("shape", SHAPES, ids=[f"{m}x{n}x{k}" for m, n, k in SHAPES])
def test_plain_ragged_all_tiles(h, op, shape):
    from paper_2109_13406_amd import binding as b
    m, n, k = shape
    for dist in ("uniform", "wide"):
        case = W.gemm_case(100 + m + n + k, op[0], op[1], m, n, k, dist=dist)
        O = gemm_oracle(case)
        for tile in range(b.mpdd_tile_count()):
            info, G = gemm_gpu(h, case, opts=dict(algo=b.MPDD_PLAIN, tile_id=tile, splitk=1))
            assert info == 0
            r = compare_full(f"ragged {op} {m}x{n}x{k} {dist} tile{tile}", G, O, m, n, k,
                             case["ldc"], C0=case["C"], case=case)
            assert r <= RATIO_MAX


@pytest.mark.parametrize("op", W.OPS)
def test_accurate_is_bit_identical_to_oracle(h, op):
    """The accurate form runs the oracle's own published steps in the same
    order (dd product, accurate dd add, increasing k; alpha then beta), so
    its result must equal the oracle's bit for bit."""
    from paper_2109_13406_amd import binding as b
    for (m, n, k) in [(97, 131, 77), (33, 17, 129), (5, 3, 1)]:
        case = W.gemm_case(200 + m, op[0], op[1], m, n, k, dist="wide")
        O = gemm_oracle(case)
        for tile in range(b.mpdd_tile_count()):
            info, G = gemm_gpu(h, case, opts=dict(algo=b.MPDD_PLAIN_ACCURATE, tile_id=tile,
                                                  splitk=1))
            assert info == 0
            assert np.array_equal(bits(G[0]), bits(O[0])), (op, m, n, k, tile)
            assert np.array_equal(bits(G[1]), bits(O[1])), (op, m, n, k, tile)
    log(f"PARITY accurate {op} bit-identical")


@pytest.mark.parametrize("splitk", [2, 4, 8])
def test_splitk(h, splitk):
    from paper_2109_13406_amd import binding as b
    for op in W.OPS:
        case = W.gemm_case(300 + splitk, op[0], op[1], 70, 9, 1000, dist="wide")
        O = gemm_oracle(case)
        for tile in (0, 2, 4):
            info, G = gemm_gpu(h, case, opts=dict(algo=b.MPDD_PLAIN, tile_id=tile, splitk=splitk))
            assert info == 0
            r = compare_full(f"splitk{splitk} {op} 70x9x1000 tile{tile}", G, O, 70, 9, 1000,
                             case["ldc"], C0=case["C"], case=case)
            assert r <= RATIO_MAX


def test_beta_zero_does_not_read_c(h):
    for op in W.OPS:
        case = W.gemm_case(400, op[0], op[1], 45, 38, 20, beta_zero=True, c_nan=True)
        O = gemm_oracle(case)
        info, G = gemm_gpu(h, case)
        assert info == 0
        r = compare_full(f"beta0 {op}", G, O, 45, 38, 20, case["ldc"], C0=case["C"],
                         case=case)
        assert r <= RATIO_MAX


def test_alpha_zero_and_k_zero(h):
    from paper_2109_13406_amd import binding as b
    import torch
    # alpha = 0: A and B are not read (NULL pointers), C = beta * C, as the oracle
    for beta_zero in (False, True):
        case = W.gemm_case(500, "N", "T", 31, 29, 7, beta_zero=beta_zero, c_nan=beta_zero)
        case["alpha"] = (0.0, 0.0)
        O = gemm_oracle(case)
        C = dev(case["C"])
        info = b.mpdd_Rgemm(h, "N", "T", 31, 29, 7, (0.0, 0.0), (None, None), case["lda"],
                            (None, None), case["ldb"], case["beta"], C, case["ldc"])
        assert info == 0
        G = host(C)
        assert np.array_equal(bits(G[0]), bits(O[0])) and np.array_equal(bits(G[1]), bits(O[1]))
    # k = 0
    case = W.gemm_case(501, "T", "N", 31, 29, 1)
    case["k"] = 0
    O = gemm_oracle(case)
    C = dev(case["C"])
    info = b.mpdd_Rgemm(h, "T", "N", 31, 29, 0, case["alpha"], (None, None), 1, (None, None), 1,
                        case["beta"], C, case["ldc"])
    assert info == 0
    G = host(C)
    assert np.array_equal(bits(G[0]), bits(O[0])) and np.array_equal(bits(G[1]), bits(O[1]))


def test_quick_returns_leave_c_untouched(h):
    from paper_2109_13406_amd import binding as b
    case = W.gemm_case(600, "N", "N", 20, 20, 20, c_nan=True)
    for (m, n, k, al, be) in ((0, 20, 20, case["alpha"], case["beta"]),
                              (20, 0, 20, case["alpha"], case["beta"]),
                              (20, 20, 20, (0.0, 0.0), (1.0, 0.0)),
                              (20, 20, 0, case["alpha"], (1.0, 0.0))):
        C = dev(case["C"])
        info = b.mpdd_Rgemm(h, "N", "N", m, n, k, al, dev(case["A"]), case["lda"],
                            dev(case["B"]), case["ldb"], be, C, case["ldc"])
        assert info == 0
        G = host(C)
        assert np.array_equal(bits(G[0]), bits(case["C"][0]))
        assert np.array_equal(bits(G[1]), bits(case["C"][1]))


def test_invalid_argument_enqueues_nothing(h):
    from paper_2109_13406_amd import binding as b
    case = W.gemm_case(700, "N", "N", 8, 8, 8, c_nan=True)
    C = dev(case["C"])
    info = b.mpdd_Rgemm(h, "N", "N", 8, 8, 8, case["alpha"], dev(case["A"]), 7, dev(case["B"]),
                        case["ldb"], case["beta"], C, case["ldc"])
    assert info == 8
    G = host(C)
    assert np.array_equal(bits(G[0]), bits(case["C"][0]))


SYRK_SHAPES = [(1, 1), (97, 45), (130, 1), (64, 200), (33, 7)]
SQUARE_TILES = (0, 1, 2, 4)      # tile-table entries with BM == BN


@pytest.mark.parametrize("uplo", "UL")
@pytest.mark.parametrize("trans", "NT")
@pytest.mark.parametrize("shape", SYRK_SHAPES, ids=[f"{n}x{k}" for n, k in SYRK_SHAPES])
def test_syrk_ragged(h, uplo, trans, shape):
    from paper_2109_13406_amd import binding as b
    n, k = shape
    for beta_zero in (False, True):
        case = W.syrk_case(800 + n + k, uplo, trans, n, k, dist="wide", beta_zero=beta_zero)
        O = syrk_oracle(case)
        for tile in SQUARE_TILES:
            info, G = syrk_gpu(h, case, opts=dict(algo=b.MPDD_PLAIN, tile_id=tile, splitk=1))
            assert info == 0
            r = compare_full(f"syrk {uplo}{trans} {n}x{k} b0={beta_zero} tile{tile}", G, O, n, n,
                             k, case["ldc"], tri=uplo, C0=case["C"], case=case)
            assert r <= RATIO_MAX
            info, G = syrk_gpu(h, case, opts=dict(algo=b.MPDD_PLAIN_ACCURATE, tile_id=tile,
                                                  splitk=1))
            assert info == 0
            assert np.array_equal(bits(G[0]), bits(O[0])) and np.array_equal(bits(G[1]), bits(O[1]))


@pytest.mark.parametrize("splitk", [2, 4, 0])
@pytest.mark.parametrize("uplo", "UL")
def test_syrk_splitk(h, uplo, splitk):
    """k-split Rsyrk (scratch partials over the triangle's tiles, masked
    reduce): within tolerance, opposite triangle and padding untouched; 0 is
    the automatic choice, which splits a small triangle with a long k."""
    from paper_2109_13406_amd import binding as b
    for trans in "NT":
        for (n, k) in ((70, 3000), (64, 2048), (130, 1100)):
            case = W.syrk_case(850 + n + k, uplo, trans, n, k, dist="wide")
            O = syrk_oracle(case)
            for tile in (0, 2, 4):
                info, G = syrk_gpu(h, case, opts=dict(algo=b.MPDD_PLAIN, tile_id=tile,
                                                      splitk=splitk))
                assert info == 0
                r = compare_full(f"syrk splitk{splitk} {uplo}{trans} {n}x{k} tile{tile}", G, O,
                                 n, n, k, case["ldc"], tri=uplo, C0=case["C"],
                                 case=case)
                assert r <= RATIO_MAX


def test_deterministic(h):
    case = W.gemm_case(900, "T", "T", 150, 140, 300)
    _, G1 = gemm_gpu(h, case)
    _, G2 = gemm_gpu(h, case)
    assert np.array_equal(bits(G1[0]), bits(G2[0])) and np.array_equal(bits(G1[1]), bits(G2[1]))


@pytest.mark.parametrize("n", [1024, 8192])
@pytest.mark.parametrize("uplo", "UL")
def test_syrk_triangle_coverage(h, uplo, n):
    """Every tile of the triangle is computed exactly once and nothing outside
    it is written, for the launch orders of triangles whose tile count is a
    multiple of 8 (8 x 8 blocks; at 8192 and 64-wide tiles, 128 tiles a side,
    each XCD's share of the blocks): full comparison with a short k."""
    from paper_2109_13406_amd import binding as b
    k = 8
    case = W.syrk_case(870 + n, uplo, "N", n, k, dist="wide")
    O = syrk_oracle(case)
    for tile in (2, 4):                  # 32- and 64-wide square tiles
        info, G = syrk_gpu(h, case, opts=dict(algo=b.MPDD_PLAIN, tile_id=tile, splitk=1))
        assert info == 0
        r = compare_full(f"syrk coverage {uplo}N {n}x{k} tile{tile}", G, O, n, n, k,
                         case["ldc"], tri=uplo, C0=case["C"], case=case)
        assert r <= RATIO_MAX
        del G


def test_bad_tile_with_automatic_split(h):
    """An out-of-range tile-table entry is rejected (not dereferenced) also
    when the k-split is left to the library."""
    from paper_2109_13406_amd import binding as b
    case = W.gemm_case(905, "N", "N", 40, 30, 50)
    for split in (0, 1):
        info, _ = gemm_gpu(h, case, opts=dict(algo=b.MPDD_PLAIN, tile_id=99, splitk=split))
        assert info == b.MPDD_ERR_UNSUPPORTED
    info, _ = syrk_gpu(h, W.syrk_case(906, "U", "N", 40, 50),
                       opts=dict(algo=b.MPDD_PLAIN, tile_id=99, splitk=0))
    assert info == b.MPDD_ERR_UNSUPPORTED


def test_binding_rejects_short_buffers(h):
    """A device plane shorter than the operand it must hold is refused by the
    binding before any kernel runs (the kernels cannot bounds-check a plain
    pointer); C is left untouched."""
    import torch
    from paper_2109_13406_amd import binding as b
    m = n = k = 64
    A = tuple(torch.zeros(64 * 64, dtype=torch.float64, device="cuda") for _ in range(2))
    Bs = tuple(torch.zeros(64 * 63, dtype=torch.float64, device="cuda") for _ in range(2))
    C = tuple(torch.full((64 * 64,), 7.0, dtype=torch.float64, device="cuda") for _ in range(2))
    with pytest.raises(ValueError, match="touches"):
        b.mpdd_Rgemm(h, "N", "N", m, n, k, 1.0, A, 64, Bs, 64, 0.0, C, 64)
    with pytest.raises(ValueError, match="touches"):
        b.mpdd_Rsyrk(h, "U", "N", 64, 64, 1.0, A, 64, 0.0, Bs, 64)
    with pytest.raises(ValueError, match="contiguous"):
        b.mpdd_Rgemm(h, "N", "N", 32, 32, 32, 1.0, tuple(x.view(64, 64)[:, :32] for x in A), 64,
                     A, 64, 0.0, C, 64)
    torch.cuda.synchronize()
    assert bool((C[0] == 7.0).all()) and bool((C[1] == 7.0).all())
    # alpha = 0, beta = 1: nothing is touched, so nothing is checked
    assert b.mpdd_Rgemm(h, "N", "N", m, n, k, 0.0, Bs, 64, Bs, 64, 1.0, C, 64) == 0

"""GPU parity of the blocked dd Cholesky Rpotrf (through the C ABI) against
the CPU oracle (the unblocked column-by-column factorisation): factors agree
normwise within 8 n 2^-104 on the well-conditioned seeded SPD inputs, the
residual ||L L^T - A|| (formed in dd by the oracle) is within LAPACK's test
threshold, the opposite triangle and padding rows are untouched, and the
info codes (argument errors, first non-positive pivot inside a block, at a
block boundary, in a later block) equal the oracle's exactly."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import dev, host, log
from oracle.compare import EPS_DD, bits

pytestmark = pytest.mark.gpu

THRESH = 30.0     # LAPACK's test-ratio threshold


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available()
    from paper_2109_13406_amd import binding as b
    handle = b.mpdd_create()
    yield handle
    torch.cuda.synchronize()
    b.mpdd_destroy(handle)


def tri_idx(n, ld, uplo):
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = (i >= j) if uplo == "L" else (i <= j)
    return (i + j * ld)[keep]


def residual_ratio(F, A, n, ld, uplo):
    """||op(F) op(F)^T - A||_F / (n ||A||_F 2^-104) on the stored triangle, the
    product formed by the dd oracle (Rsyrk of the factor)."""
    # factor as a full matrix with zeros outside its triangle
    Fh = np.zeros(n * n)
    Fl = np.zeros(n * n)
    idx = tri_idx(n, ld, uplo)
    idn = tri_idx(n, n, uplo)
    Fh[idn] = F[0][idx]
    Fl[idn] = F[1][idx]
    P = (np.zeros(n * n), np.zeros(n * n))
    trans = "N" if uplo == "L" else "T"        # L L^T  or  U^T U
    assert oracle.rsyrk(uplo, trans, n, n, (1.0, 0.0), (Fh, Fl), n, (0.0, 0.0), P, n) == 0
    d = (P[0][idn] - A[0][idx]) + (P[1][idn] - A[1][idx])
    return float(np.linalg.norm(d) / (n * np.linalg.norm(A[0][idx]) * EPS_DD))


def run_gpu(h, c, nb=0):
    from paper_2109_13406_amd import binding as b
    A = dev(c["A"])
    rc, info = b.mpdd_Rpotrf(h, c["uplo"], c["n"], A, c["lda"], nb=nb)
    assert rc == 0
    return info, host(A)


def run_oracle(c):
    O = (c["A"][0].copy(), c["A"][1].copy())
    return oracle.rpotrf(c["uplo"], c["n"], O, c["lda"]), O


SIZES = [1, 5, 63, 64, 65, 128, 129, 300]


@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("n", SIZES)
def test_potrf_vs_oracle(h, uplo, n):
    for nb in (0, 32, 7):
        c = W.spd_case(5000 + n, n, uplo)
        io, O = run_oracle(c)
        ig, G = run_gpu(h, c, nb)
        assert io == 0 and ig == 0
        idx = tri_idx(n, c["lda"], uplo)
        d = (G[0][idx] - O[0][idx]) + (G[1][idx] - O[1][idx])
        r = float(np.linalg.norm(d) / np.linalg.norm(O[0][idx]) / (n * EPS_DD))
        res = residual_ratio(G, c["A"], n, c["lda"], uplo)
        log(f"PARITY potrf {uplo} n={n} nb={nb}: factor ratio {r:.4g}, residual {res:.4g}")
        assert r <= 8.0, (uplo, n, nb, r)
        assert res <= THRESH, (uplo, n, nb, res)
        rest = np.ones(G[0].shape[0], bool)
        rest[idx] = False
        assert np.array_equal(bits(G[0])[rest], bits(c["A"][0])[rest])
        assert np.array_equal(bits(G[1])[rest], bits(c["A"][1])[rest])


@pytest.mark.parametrize("uplo", "LU")
def test_potrf_info_not_positive_definite(h, uplo):
    n = 300
    for k in (1, 50, 64, 65, 129, 257, 300):
        for nb in (0, 64):
            c = W.spd_case(5100 + k, n, uplo, fail_at=k)
            io, _ = run_oracle(c)
            ig, _ = run_gpu(h, c, nb)
            assert io == k and ig == k, (uplo, k, nb, io, ig)


def test_potrf_argument_errors(h):
    from paper_2109_13406_amd import binding as b
    c = W.spd_case(5200, 4, "L")
    A = dev(c["A"])
    assert b.mpdd_Rpotrf(h, "X", 4, A, c["lda"]) == (0, -1)
    assert b.mpdd_Rpotrf(h, "L", -1, A, c["lda"]) == (0, -2)
    assert b.mpdd_Rpotrf(h, "L", 4, A, 3) == (0, -4)
    assert b.mpdd_Rpotrf(h, "L", 0, A, 1) == (0, 0)
    assert b.mpdd_Rpotrf(h, "L", 4, A, c["lda"], nb=65) == (b.MPDD_ERR_UNSUPPORTED, 0)
    G = host(A)
    assert np.array_equal(bits(G[0]), bits(c["A"][0]))


@pytest.mark.parametrize("uplo", "LU")
def test_potrf_1024(h, uplo):
    n = 1024
    c = W.spd_case(5300, n, uplo)
    io, O = run_oracle(c)
    ig, G = run_gpu(h, c)
    assert io == 0 and ig == 0
    idx = tri_idx(n, c["lda"], uplo)
    d = (G[0][idx] - O[0][idx]) + (G[1][idx] - O[1][idx])
    r = float(np.linalg.norm(d) / np.linalg.norm(O[0][idx]) / (n * EPS_DD))
    log(f"PARITY potrf {uplo} n={n}: factor ratio {r:.4g}")
    assert r <= 8.0

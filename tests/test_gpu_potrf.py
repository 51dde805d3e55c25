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


def run_gpu(h, c, nb=0, opts=None):
    from paper_2109_13406_amd import binding as b
    A = dev(c["A"])
    rc, info = b.mpdd_Rpotrf(h, c["uplo"], c["n"], A, c["lda"], nb=nb, opts=opts)
    assert rc == 0
    return info, host(A)


# right-looking form with split-form (INT8, 12 slices) trailing updates
SPLIT = dict(algo=1, nslices=12)
CRT = dict(algo=5, nslices=26)      # modular split form, the benchmark's 26 moduli


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
@pytest.mark.parametrize("n,nb", [(65, 0), (1100, 0), (1100, 32), (2100, 48)])
def test_potrf_split_updates_vs_oracle(h, uplo, n, nb):
    """Right-looking Rpotrf over 1024-column panels whose trailing updates
    are split-form Rsyrk calls (INT8 with 12 slices, FP64 with 5, modular
    with 26 moduli): the
    factor within 8 n 2^-104 of the oracle's, the residual within LAPACK's
    threshold (formed by the oracle up to n = 1100), nothing outside the
    triangle touched; n = 1100 takes two panels (the last ragged), n = 2100
    three, n = 65 one."""
    for opts in (SPLIT, dict(algo=2, nslices=5), CRT):
        c = W.spd_case(5500 + n, n, uplo)
        io, O = run_oracle(c)
        ig, G = run_gpu(h, c, nb=nb, opts=opts)
        assert io == 0 and ig == 0
        idx = tri_idx(n, c["lda"], uplo)
        d = (G[0][idx] - O[0][idx]) + (G[1][idx] - O[1][idx])
        r = float(np.linalg.norm(d) / np.linalg.norm(O[0][idx]) / (n * EPS_DD))
        res = residual_ratio(G, c["A"], n, c["lda"], uplo) if n <= 1100 else 0.0
        log(f"PARITY potrf split {opts['algo']} {uplo} n={n} nb={nb}: factor ratio {r:.4g}, "
            f"residual {res:.4g}")
        assert r <= 8.0, (uplo, n, opts, r)
        assert res <= THRESH, (uplo, n, opts, res)
        rest = np.ones(G[0].shape[0], bool)
        rest[idx] = False
        assert np.array_equal(bits(G[0])[rest], bits(c["A"][0])[rest])
        assert np.array_equal(bits(G[1])[rest], bits(c["A"][1])[rest])


@pytest.mark.parametrize("uplo", "LU")
def test_potrf_split_updates_info(h, uplo):
    """Failing pivots in the first and second panel and at the panel
    boundary (1024 columns with nb = 64 and 32) give the oracle's info; an
    unknown algo is rejected."""
    from paper_2109_13406_amd import binding as b
    n = 1100
    for k in (1, 300, 512, 513, 1024, 1025, 1100):
        for nb in (0, 32):
            c = W.spd_case(5600 + k, n, uplo, fail_at=k)
            io, _ = run_oracle(c)
            ig, _ = run_gpu(h, c, nb=nb, opts=SPLIT)
            assert io == k and ig == k, (uplo, k, nb, io, ig)
    c = W.spd_case(5700, 8, uplo)
    rc, _ = b.mpdd_Rpotrf(h, uplo, 8, dev(c["A"]), c["lda"], opts=dict(algo=3))
    assert rc == b.MPDD_ERR_ARG


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


@pytest.mark.parametrize("form", ["plain", "split", "crt"])
@pytest.mark.parametrize("uplo", "LU")
def test_potrf_8192_sampled(h, uplo, form):
    """The benchmarked size (n = 8192, ld = 8195), checked where the oracle can
    follow it: the leading 256 x 256 block equals the oracle's factor of the
    leading principal submatrix, the first 256 entries of sampled later rows
    equal the last row of the oracle's factor of the principal submatrix on
    indices [0, 256) + {i} (a Cholesky factor's row i, columns < c, depends only
    on A's leading c columns), and sampled entries of L L^T - A, formed in dd by
    the oracle's Rgemm, are within LAPACK's threshold of the componentwise
    backward-error bound n 2^-104 sqrt(A(i,i) A(j,j))."""
    import torch
    from paper_2109_13406_amd import binding as b
    n, n0 = 8192, 256
    c = W.spd_case_device(5400, n, uplo)
    ld = c["lda"]

    def lower_view(planes):
        # X(r, l) of the lower view as an (n, n) torch view: 'L' A(r, l), 'U' A(l, r)
        v = [p[: n * ld].view(n, ld)[:, :n] for p in planes]     # v[j, i] = A(i, j)
        return [x.t() for x in v] if uplo == "L" else v

    A0 = lower_view(c["A"])
    A_lead = [x[:n0, :n0].cpu().numpy() for x in A0]
    rng = np.random.default_rng(5401)
    rows = np.sort(rng.choice(np.arange(n0, n), 8, replace=False))
    A_rows = [[x[i, :n0].cpu().numpy() for x in A0] for i in rows]
    A_rowdiag = [[float(x[i, i]) for x in A0] for i in rows]
    ii = rng.integers(0, n, 48)
    jj = (rng.random(48) * (ii + 1)).astype(np.int64)
    ii = np.concatenate([ii, [n - 1, n - 1, n - 1]])
    jj = np.concatenate([jj, [0, n - 2, n - 1]])
    A_ij = [(float(A0[0][i, j]), float(A0[1][i, j])) for i, j in zip(ii, jj)]
    diag = A0[0].diagonal().cpu().numpy().copy()

    rc, info = b.mpdd_Rpotrf(h, uplo, n, c["A"], ld,
                             opts={"plain": None, "split": SPLIT, "crt": CRT}[form])
    torch.cuda.synchronize()
    assert rc == 0 and info == 0
    L = lower_view(c["A"])

    def lower_tri(M):
        # oracle layout of an m x m lower-view matrix M (numpy, [r, l])
        m = M.shape[0]
        return np.ascontiguousarray(M.T if uplo == "L" else M).reshape(-1).copy()

    # leading block
    O = (lower_tri(A_lead[0]), lower_tri(A_lead[1]))
    assert oracle.rpotrf(uplo, n0, O, n0) == 0
    G = [x[:n0, :n0].cpu().numpy() for x in L]
    Gf = (lower_tri(G[0]), lower_tri(G[1]))
    idx = tri_idx(n0, n0, uplo)
    d = (Gf[0][idx] - O[0][idx]) + (Gf[1][idx] - O[1][idx])
    r = float(np.linalg.norm(d) / np.linalg.norm(O[0][idx]) / (n0 * EPS_DD))
    log(f"PARITY potrf {form} {uplo} n={n} leading {n0}: factor ratio {r:.4g}")
    assert r <= 8.0

    # sampled rows, first n0 columns
    for t, i in enumerate(rows):
        S = [np.zeros((n0 + 1, n0 + 1)) for _ in range(2)]
        for p in range(2):
            S[p][:n0, :n0] = np.tril(A_lead[p])
            S[p][n0, :n0] = A_rows[t][p]
            S[p][n0, n0] = A_rowdiag[t][p]
        O = (lower_tri(S[0]), lower_tri(S[1]))
        assert oracle.rpotrf(uplo, n0 + 1, O, n0 + 1) == 0
        og = [O[p].reshape(n0 + 1, n0 + 1) for p in range(2)]   # [col, row] for L, [row, col] for U
        orow = [(og[p][:n0, n0] if uplo == "L" else og[p][n0, :n0]) for p in range(2)]
        grow = [x[i, :n0].cpu().numpy() for x in L]
        d = (grow[0] - orow[0]) + (grow[1] - orow[1])
        r = float(np.linalg.norm(d) / np.linalg.norm(orow[0]) / (n0 * EPS_DD))
        log(f"PARITY potrf {form} {uplo} n={n} row {i} cols <{n0}: ratio {r:.4g}")
        assert r <= 8.0, (i, r)

    # sampled residual entries (L L^T - A)(i, j), i >= j
    worst = 0.0
    for (i, j), (ah, al) in zip(zip(ii, jj), A_ij):
        kk = int(j) + 1
        Li = [np.ascontiguousarray(x[int(i), :kk].cpu().numpy()) for x in L]
        Lj = [np.ascontiguousarray(x[int(j), :kk].cpu().numpy()) for x in L]
        C = (np.array([ah]), np.array([al]))
        assert oracle.rgemm("N", "T", 1, 1, kk, (1.0, 0.0), Li, 1, Lj, 1, (-1.0, 0.0), C, 1) == 0
        res = abs(C[0][0] + C[1][0]) / (n * EPS_DD * np.sqrt(diag[i] * diag[j]))
        worst = max(worst, res)
    log(f"PARITY potrf {form} {uplo} n={n}: worst sampled residual ratio {worst:.4g}")
    assert worst <= THRESH

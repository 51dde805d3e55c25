"""GPU parity of the complex dd Cgemm (through the C ABI) against the CPU
oracle: the manual's worked Cgemm example, ragged shapes in all nine op
combinations, BLAS semantics (beta = 0 with NaN C, alpha = 0, k = 0, quick
returns, untouched padding, info codes), and a 2048-size product checked on
sampled rows and columns.

The error metric is the real one applied to all 2mn real components:
||dC||_F / ||C_oracle||_F <= 8 k 2^-104."""
import numpy as np
import pytest

import oracle
import pins
import workloads as W
from gpu_util import csub, log, take
from oracle.compare import RATIO_MAX, bits, ratio

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


def dev4(planes):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in planes)


def host4(planes):
    import torch
    torch.cuda.synchronize()
    return tuple(x.cpu().numpy() for x in planes)


def cgemm_gpu(h, c, opts=None):
    from paper_2109_13406_amd import binding as b
    C = dev4(c["C"])
    args = (c["transa"], c["transb"], c["m"], c["n"], c["k"], c["alpha"], dev4(c["A"]), c["lda"],
            dev4(c["B"]), c["ldb"], c["beta"], C, c["ldc"])
    if opts is None:
        info = b.mpdd_Cgemm(h, *args)
    else:
        info = b.mpdd_Cgemm_ex(h, opts, *args)
    return info, host4(C)


def cgemm_oracle(c):
    O = tuple(p.copy() for p in c["C"])
    assert oracle.cgemm(c["transa"], c["transb"], c["m"], c["n"], c["k"], c["alpha"], c["A"],
                        c["lda"], c["B"], c["ldb"], c["beta"], O, c["ldc"]) == 0
    return O


def cratio(G, O, idx, k):
    """Normwise ratio over the real and imaginary parts of the entries idx."""
    gh = np.concatenate([G[0][idx], G[2][idx]])
    gl = np.concatenate([G[1][idx], G[3][idx]])
    oh = np.concatenate([O[0][idx], O[2][idx]])
    ol = np.concatenate([O[1][idx], O[3][idx]])
    return ratio(gh, gl, oh, ol, k)


def stored(m, n, ldc):
    i, j = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    return (i + j * ldc).ravel()


def compare(label, G, O, C0, m, n, k, ldc):
    idx = stored(m, n, ldc)
    r = cratio(G, O, idx, k)
    log(f"PARITY cgemm {label}: ratio {r:.4g}")
    rest = np.ones(G[0].shape[0], bool)
    rest[idx] = False
    for g, c0 in zip(G, C0):
        assert np.array_equal(bits(g)[rest], bits(c0)[rest]), label
    return r


def test_worked_example(h):
    """The manual's demo with binary64 inputs: every op form of the GPU result
    is within the dd error bound of the printed 64-digit answer, and within
    the normwise tolerance of the oracle."""
    from fractions import Fraction
    ex = pins.read_cgemm_example()
    todd = lambda s: (float(s), 0.0)       # noqa: E731
    Ap, Bp, Cp = (pins._cplanes(ex[k], todd) for k in ("A", "B", "C"))
    alpha = (todd(ex["alpha"][0]), todd(ex["alpha"][1]))
    beta = (todd(ex["beta"][0]), todd(ex["beta"][1]))
    ans = [[(Fraction(r), Fraction(i)) for r, i in row] for row in ex["ANSWER_BINARY64"]]

    def prep(P, t):
        M = [p.reshape(3, 3, order="F") for p in P]
        if t != "N":
            M = [m.T for m in M]
        if t == "C":
            M[2], M[3] = -M[2], -M[3]
        return tuple(pins.colmajor(m) for m in M)
    for ta, tb in W.COPS:
        c = dict(transa=ta, transb=tb, m=3, n=3, k=3, alpha=alpha, beta=beta, A=prep(Ap, ta),
                 lda=3, B=prep(Bp, tb), ldb=3, C=tuple(p.copy() for p in Cp), ldc=3)
        info, G = cgemm_gpu(h, c)
        assert info == 0
        O = cgemm_oracle(c)
        assert compare(f"worked example {ta}{tb}", G, O, Cp, 3, 3, 3, 3) <= RATIO_MAX
        for i in range(3):
            for j in range(3):
                o = i + 3 * j
                got = (pins.F(G[0][o], G[1][o]), pins.F(G[2][o], G[3][o]))
                for q in range(2):
                    # |answer| is within 400 here; 2^-90 relative is far below binary64
                    assert abs(got[q] - ans[i][j][q]) <= Fraction(400, 2 ** 90), (ta, tb, i, j)


SHAPES = [(1, 1, 1), (97, 131, 77), (65, 1, 300), (130, 70, 33), (200, 190, 1)]


@pytest.mark.parametrize("form", ["4M", "3M", "split", "crt"])
@pytest.mark.parametrize("op", W.COPS, ids=[a + b for a, b in W.COPS])
def test_cgemm_ragged(h, op, form):
    from paper_2109_13406_amd import binding as b
    opts = {"4M": None, "3M": dict(algo=b.MPDD_COMPLEX_3M),
            "split": dict(algo=b.MPDD_OZAKI_I8, nslices=22),
            "crt": dict(algo=b.MPDD_OZAKI_CRT, nslices=30)}[form]
    for (m, n, k) in SHAPES:
        for dist in ("uniform", "wide"):
            c = W.cgemm_case(4000 + m + k, op[0], op[1], m, n, k, dist=dist)
            O = cgemm_oracle(c)
            info, G = cgemm_gpu(h, c, opts)
            assert info == 0
            r = compare(f"{form} {op} {m}x{n}x{k} {dist}", G, O, c["C"], m, n, k, c["ldc"])
            assert r <= RATIO_MAX, (form, op, m, n, k, dist, r)


def test_cgemm_3m_options(h):
    """The three-product form at 512^3 (k-split and tile choices passed on),
    and an algo Cgemm does not take rejected before any work."""
    from paper_2109_13406_amd import binding as b
    c = W.cgemm_case(W.BASE_SEED + 5, "C", "N", 512, 512, 512)
    O = cgemm_oracle(c)
    for tile in (-1, 2):
        info, G = cgemm_gpu(h, c, dict(algo=b.MPDD_COMPLEX_3M, tile_id=tile))
        assert info == 0
        assert compare(f"3M 512^3 CN tile{tile}", G, O, c["C"], 512, 512, 512,
                       c["ldc"]) <= RATIO_MAX
    info, G = cgemm_gpu(h, W.cgemm_case(1, "N", "N", 4, 4, 4),
                        dict(algo=b.MPDD_PLAIN_ACCURATE))
    assert info == b.MPDD_ERR_ARG


def test_cgemm_semantics(h):
    from paper_2109_13406_amd import binding as b
    import torch
    z = ((0.0, 0.0), (0.0, 0.0))
    one = ((1.0, 0.0), (0.0, 0.0))
    # beta = 0: a NaN C is not read
    c = W.cgemm_case(4100, "C", "T", 45, 38, 20, beta_zero=True, c_nan=True)
    O = cgemm_oracle(c)
    info, G = cgemm_gpu(h, c)
    assert info == 0
    assert compare("beta0", G, O, c["C"], 45, 38, 20, c["ldc"]) <= RATIO_MAX
    # alpha = 0 (A, B NULL): C <- beta C, bit-identical to the oracle (same steps)
    for beta_zero in (False, True):
        c = W.cgemm_case(4101, "N", "C", 31, 29, 7, beta_zero=beta_zero, c_nan=beta_zero)
        c["alpha"] = z
        O = cgemm_oracle(c)
        C = dev4(c["C"])
        N4 = (None,) * 4
        assert b.mpdd_Cgemm(h, "N", "C", 31, 29, 7, z, N4, c["lda"], N4, c["ldb"], c["beta"], C,
                            c["ldc"]) == 0
        G = host4(C)
        for g, o in zip(G, O):
            assert np.array_equal(bits(g), bits(o)), beta_zero
    # k = 0 behaves as alpha = 0
    c = W.cgemm_case(4102, "T", "N", 17, 9, 1)
    c["k"] = 0
    O = cgemm_oracle(c)
    C = dev4(c["C"])
    assert b.mpdd_Cgemm(h, "T", "N", 17, 9, 0, c["alpha"], (None,) * 4, 1, (None,) * 4, 1,
                        c["beta"], C, c["ldc"]) == 0
    for g, o in zip(host4(C), O):
        assert np.array_equal(bits(g), bits(o))
    # quick returns leave C bit-identical; an invalid lda enqueues nothing
    c = W.cgemm_case(4103, "N", "N", 20, 20, 20, c_nan=True)
    A, B = dev4(c["A"]), dev4(c["B"])
    for (m, n, k, al, be, lda, want) in ((0, 20, 20, c["alpha"], c["beta"], c["lda"], 0),
                                         (20, 0, 20, c["alpha"], c["beta"], c["lda"], 0),
                                         (20, 20, 20, z, one, c["lda"], 0),
                                         (20, 20, 0, c["alpha"], one, c["lda"], 0),
                                         (20, 20, 20, c["alpha"], c["beta"], 19, 8)):
        C = dev4(c["C"])
        assert b.mpdd_Cgemm(h, "N", "N", m, n, k, al, A, lda, B, c["ldb"], be, C, c["ldc"]) == want
        for g, c0 in zip(host4(C), c["C"]):
            assert np.array_equal(bits(g), bits(c0))
    torch.cuda.synchronize()


@pytest.mark.parametrize("op", [("N", "N"), ("C", "N"), ("T", "C")], ids=["NN", "CN", "TC"])
def test_cgemm_512_full(h, op):
    c = W.cgemm_case(W.BASE_SEED + 5, op[0], op[1], 512, 512, 512)
    O = cgemm_oracle(c)
    info, G = cgemm_gpu(h, c)
    assert info == 0
    assert compare(f"512^3 {op}", G, O, c["C"], 512, 512, 512, c["ldc"]) <= RATIO_MAX


def test_cgemm_2048_sampled(h):
    """A 2048^3 product (tile grid, no k-split) checked on 48 x 48 sampled
    entries: the oracle runs on the gathered rows of op(A) and columns of
    op(B)."""
    n = k = 2048
    for ta, tb in (("N", "N"), ("C", "T")):
        c = W.cgemm_case(W.BASE_SEED + 6, ta, tb, n, n, k)
        info, G = cgemm_gpu(h, c)
        assert info == 0
        rng = np.random.default_rng(7)
        I = np.sort(rng.choice(n, 48, replace=False))
        J = np.sort(rng.choice(n, 48, replace=False))
        sub = csub(c, I, J)
        O = cgemm_oracle(sub)
        Gs = tuple(p[(I[:, None] + J[None, :] * c["ldc"]).ravel(order="F")] for p in G)
        r = cratio(Gs, O, np.arange(48 * 48), k)
        log(f"PARITY cgemm 2048^3 {ta}{tb} sampled 48x48: ratio {r:.4g}")
        assert r <= RATIO_MAX


def test_cgemm_4096_sampled(h):
    """The benchmarked size and inputs (4096^3 NN, device-generated operands;
    the four- and the three-product form, and the four products in the INT8
    split form with the benchmark's 12 slices and in the modular form with
    its 26 moduli) on 32 x 32 sampled entries:
    the oracle runs on the gathered rows of op(A) and columns of op(B)."""
    import torch
    from paper_2109_13406_amd import binding as b
    n = 4096
    for form, opts in (("4M", None), ("3M", dict(algo=b.MPDD_COMPLEX_3M)),
                       ("split", dict(algo=b.MPDD_OZAKI_I8, nslices=12)),
                       ("crt", dict(algo=b.MPDD_OZAKI_CRT, nslices=26))):
        c = W.cgemm_case_device(W.BASE_SEED + 5, "N", "N", n, n, n)
        rng = np.random.default_rng(11)
        I = np.sort(rng.choice(n, 32, replace=False))
        J = np.sort(rng.choice(n, 32, replace=False))
        sub = csub(c, I, J)
        args = ("N", "N", n, n, n, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"], c["beta"],
                c["C"], c["ldc"])
        info = b.mpdd_Cgemm(h, *args) if opts is None else b.mpdd_Cgemm_ex(h, opts, *args)
        torch.cuda.synchronize()
        assert info == 0
        O = cgemm_oracle(sub)
        Gs = tuple(take(p, (I[:, None] + J[None, :] * c["ldc"]).ravel(order="F")) for p in c["C"])
        r = cratio(Gs, O, np.arange(32 * 32), n)
        log(f"PARITY cgemm {n}^3 NN {form} (benchmarked inputs) sampled 32x32: ratio {r:.4g}")
        assert r <= RATIO_MAX
        del c

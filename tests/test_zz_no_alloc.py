"""The no-allocation Rgemm (mpdd_Rgemm_noalloc, k-split partials in the
library's static per-device scratch) against mpdd_Rgemm_ex, the entry point
it is a variant of, and against the CPU oracle: every call through the C ABI.

Two calls in a row, the second with a smaller input (the scratch keeps the
first call's partials), each bit-identical to mpdd_Rgemm_ex with the same
options (same kernels, same k-split) and within the normwise bound of the
oracle; an automatic split whose partials would not fit is halved (the result
equals mpdd_Rgemm_ex with that explicit split); an explicit split that does
not fit is rejected with nothing enqueued."""
import numpy as np
import pytest

import workloads as W
from gpu_util import compare_full, dev, gemm_oracle, host, log
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


def _args(case, A, B, C):
    return (case["transa"], case["transb"], case["m"], case["n"], case["k"], case["alpha"], A,
            case["lda"], B, case["ldb"], case["beta"], C, case["ldc"])


def _run(h, case, entry, opts):
    """(info, C on the host) of one call on device copies of the case."""
    from paper_2109_13406_amd import binding as b
    A, B, C = dev(case["A"]), dev(case["B"]), dev(case["C"])
    fn = b.mpdd_Rgemm_noalloc if entry == "noalloc" else b.mpdd_Rgemm_ex
    info = fn(h, opts, *_args(case, A, B, C))
    return info, host(C)


def _same_bits(G, R):
    return np.array_equal(bits(G[0]), bits(R[0])) and np.array_equal(bits(G[1]), bits(R[1]))


# (seed offset, transa, transb, m, n, k, opts): the second call of each pair is
# smaller than the first; the k-ranges make the default plan split k.
PAIRS = [
    ((1, "N", "N", 1000, 70, 3000, None), (2, "T", "N", 300, 40, 2000, None)),
    ((3, "N", "T", 513, 130, 4100, dict(splitk=8)), (4, "T", "T", 77, 65, 1500, dict(splitk=4))),
    ((5, "N", "N", 700, 90, 2600, dict(algo=3)), (6, "N", "T", 129, 33, 1200, dict(algo=3))),
]


@pytest.mark.parametrize("pair", PAIRS, ids=lambda p: f"{p[0][1]}{p[0][2]}{p[0][3]}-then-{p[1][3]}")
def test_noalloc_matches_rgemm_ex_twice(h, pair):
    for (off, ta, tb, m, n, k, opts) in pair:
        case = W.gemm_case(W.BASE_SEED + 700 + off, ta, tb, m, n, k)
        print(f"noalloc case {ta}{tb} m={m} n={n} k={k} opts={opts}", flush=True)
        info, G = _run(h, case, "noalloc", opts)
        assert info == 0
        info_ref, R = _run(h, case, "ex", opts)
        assert info_ref == 0
        assert _same_bits(G, R), f"{ta}{tb} {m}x{n}x{k} {opts}: differs from mpdd_Rgemm_ex"
        O = gemm_oracle(case)
        r = compare_full(f"noalloc {ta}{tb} {m}x{n}x{k} {opts}", G, O, m, n, k, case["ldc"],
                         C0=case["C"], case=case)
        assert r <= RATIO_MAX


def test_noalloc_auto_split_halved_to_fit(h):
    """m = n = 1100, k = 4096: the default plan splits k in 4 (16*4*m*n bytes
    of partials, more than the 64 MiB static scratch); the no-allocation call
    halves it to 2, so it equals mpdd_Rgemm_ex with splitk = 2 bit for bit,
    and an explicit splitk = 4 is rejected with C untouched."""
    import torch
    from paper_2109_13406_amd import binding as b
    from gpu_util import gather, sample_indices, sampled_oracle
    from oracle.compare import ratio
    m = n = 1100
    k = 4096
    assert 16 * 4 * m * n > b.MPDD_STATIC_SCRATCH_BYTES >= 16 * 2 * m * n
    case = W.gemm_case_device(W.BASE_SEED + 710, "N", "N", m, n, k)
    C0 = tuple(x.clone() for x in case["C"])
    same = lambda X, Y: all(torch.equal(x.view(torch.int64), y.view(torch.int64))
                            for x, y in zip(X, Y))
    print("noalloc halved split: NN 1100x1100x4096", flush=True)
    args = _args(case, case["A"], case["B"], case["C"])
    # an explicit split that does not fit: rejected, nothing enqueued
    assert b.mpdd_Rgemm_noalloc(h, dict(splitk=4), *args) == b.MPDD_ERR_SCRATCH
    torch.cuda.synchronize()
    assert same(case["C"], C0)
    # the split forms are not offered without allocation
    assert b.mpdd_Rgemm_noalloc(h, dict(algo=b.MPDD_OZAKI_I8), *args) == b.MPDD_ERR_UNSUPPORTED
    # automatic plan: halved to splitk = 2
    assert b.mpdd_Rgemm_noalloc(h, None, *args) == 0
    torch.cuda.synchronize()
    G = tuple(x.clone() for x in case["C"])
    for dst, src in zip(case["C"], C0):
        dst.copy_(src)
    assert b.mpdd_Rgemm_ex(h, dict(splitk=2), *args) == 0
    torch.cuda.synchronize()
    assert same(G, case["C"]), "halved split differs from mpdd_Rgemm_ex with splitk = 2"
    # the no-allocation result against the oracle on sampled entries
    ii, jj = sample_indices(m, n, 128, 3)
    flat = ii + jj * case["ldc"]
    cin = gather(C0, flat)
    got = gather(G, flat)
    ref = sampled_oracle("N", "N", k, case["alpha"], case["A"], case["lda"], case["B"],
                         case["ldb"], case["beta"], cin, ii, jj)
    r = ratio(got[0], got[1], ref[0], ref[1], k)
    log(f"PARITY noalloc halved split NN 1100x1100x4096 sampled({len(ii)}) ratio={r:.3g}")
    assert r <= RATIO_MAX


def test_noalloc_quick_returns_and_scale(h):
    """alpha = 0 (C = beta*C, no scratch) and the BLAS quick return, through
    the no-allocation entry point, equal mpdd_Rgemm_ex bit for bit."""
    for alpha, beta in (((0.0, 0.0), (0.75, 1e-17)), ((0.0, 0.0), (1.0, 0.0)),
                        ((0.5, 0.0), (0.0, 0.0))):
        case = W.gemm_case(W.BASE_SEED + 720, "N", "N", 90, 50, 700)
        case["alpha"], case["beta"] = alpha, beta
        info, G = _run(h, case, "noalloc", None)
        assert info == 0
        info, R = _run(h, case, "ex", None)
        assert info == 0
        assert _same_bits(G, R), (alpha, beta)

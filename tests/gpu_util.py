"""Helpers for the GPU parity tests: move seeded cases to the device, run the
HIP library through its C ABI, bring results back, compare with the oracle."""
import os
import sys

import numpy as np

import oracle
from oracle.compare import bits, ratio

RESULTS = os.environ.get("MPDD_PARITY_LOG", os.path.join(
    os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out", "parity.log"))


def log(msg):
    """One line per checked result, to stdout and the parity log."""
    print(msg, flush=True)
    try:
        os.makedirs(os.path.dirname(RESULTS), exist_ok=True)
        with open(RESULTS, "a") as f:
            f.write(msg + "\n")
    except OSError:
        pass


def dev(pair):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in pair)


def host(pair):
    import torch
    torch.cuda.synchronize()
    return tuple(x.cpu().numpy() for x in pair)


def gemm_gpu(h, case, opts=None, stream=None):
    """Run mpdd_Rgemm(_ex) on device copies of a case; returns (info, C host)."""
    from paper_2109_13406_amd import binding as b
    A, B, C = dev(case["A"]), dev(case["B"]), dev(case["C"])
    args = (case["transa"], case["transb"], case["m"], case["n"], case["k"], case["alpha"], A,
            case["lda"], B, case["ldb"], case["beta"], C, case["ldc"])
    if opts is None:
        info = b.mpdd_Rgemm(h, *args, stream=stream)
    else:
        info = b.mpdd_Rgemm_ex(h, opts, *args, stream=stream)
    return info, host(C)


def syrk_gpu(h, case, opts=None, stream=None):
    from paper_2109_13406_amd import binding as b
    A, C = dev(case["A"]), dev(case["C"])
    args = (case["uplo"], case["trans"], case["n"], case["k"], case["alpha"], A, case["lda"],
            case["beta"], C, case["ldc"])
    if opts is None:
        info = b.mpdd_Rsyrk(h, *args, stream=stream)
    else:
        info = b.mpdd_Rsyrk_ex(h, opts, *args, stream=stream)
    return info, host(C)


def gemm_oracle(case):
    C = (case["C"][0].copy(), case["C"][1].copy())
    info = oracle.rgemm(case["transa"], case["transb"], case["m"], case["n"], case["k"],
                        case["alpha"], case["A"], case["lda"], case["B"], case["ldb"],
                        case["beta"], C, case["ldc"])
    assert info == 0
    return C


def syrk_oracle(case):
    C = (case["C"][0].copy(), case["C"][1].copy())
    info = oracle.rsyrk(case["uplo"], case["trans"], case["n"], case["k"], case["alpha"],
                        case["A"], case["lda"], case["beta"], C, case["ldc"])
    assert info == 0
    return C


def entries_mask(m, n, ldc, tri=None):
    """Flat indices of the stored entries (or of one triangle) of an m x n C."""
    i, j = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    sel = np.ones_like(i, dtype=bool)
    if tri == "U":
        sel = i <= j
    elif tri == "L":
        sel = i >= j
    return (i + j * ldc)[sel]


def compare_full(name, G, O, m, n, k, ldc, tri=None, check_rest=True, C0=None):
    """Ratio over the stored entries; everything else bit-identical to C0."""
    idx = entries_mask(m, n, ldc, tri)
    r = ratio(G[0][idx], G[1][idx], O[0][idx], O[1][idx], k)
    log(f"PARITY {name} ratio={r:.3g}")
    if check_rest and C0 is not None:
        rest = np.ones(G[0].shape[0], bool)
        rest[idx] = False
        assert np.array_equal(bits(G[0])[rest], bits(C0[0])[rest]), f"{name}: untouched region changed"
        assert np.array_equal(bits(G[1])[rest], bits(C0[1])[rest]), f"{name}: untouched region changed"
    return r


def sample_indices(m, n, count, seed, tri=None):
    """Random entries plus the corners and edges of the matrix (ragged tails
    and tile boundaries live there)."""
    rng = np.random.default_rng(seed)
    ii = list(rng.integers(0, m, count))
    jj = list(rng.integers(0, n, count))
    for i in (0, m - 1, m // 2):
        for j in (0, n - 1, n // 2, min(n - 1, 63), min(n - 1, 64)):
            ii.append(i)
            jj.append(j)
    ii, jj = np.array(ii), np.array(jj)
    if tri == "U":
        sw = ii > jj
        ii[sw], jj[sw] = jj[sw].copy(), ii[sw].copy()
    elif tri == "L":
        sw = ii < jj
        ii[sw], jj[sw] = jj[sw].copy(), ii[sw].copy()
    return ii, jj

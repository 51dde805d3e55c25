"""GPU parity at the full workload sizes, in the launch configuration the
benchmark uses (default tile / k-split choice), checked against the oracle on
sampled entries (random ones plus corners, edges and tile boundaries):

* plain Rgemm, four op combinations x m = n = k in {1024, 2048, 4096, 8192},
  plus 4096 x 4096 x 256 and the skinny 8192 x 64 x 8192 (k-split);
  leading dimensions padded to 64*ceil(rows/64) + 3;
* plain Rsyrk, uplo x trans x n in {2048, 8192} x k in {512, 8192}, once with
  beta = 0 and C filled with a NaN sentinel, once with a random beta; the
  opposite triangle (and the padding) must come back bit-identical.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import log, sampled_gemm_check, sampled_syrk_check
from oracle.compare import RATIO_MAX

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    from paper_2109_13406_amd import binding as b
    handle = b.mpdd_create()
    yield handle
    torch.cuda.synchronize()
    b.mpdd_destroy(handle)


@pytest.fixture(autouse=True)
def _free():
    yield
    import torch
    torch.cuda.empty_cache()


@pytest.mark.parametrize("run", W.config1_runs(), ids=lambda r: f"{r[0]}{r[1]}-{r[2]}x{r[3]}x{r[4]}")
def test_config1_rgemm(h, run):
    ta, tb, m, n, k = run
    case = W.gemm_case_device(W.BASE_SEED + 1 + m + k, ta, tb, m, n, k)
    r = sampled_gemm_check(h, f"config1 {ta}{tb} {m}x{n}x{k}", case, seed=m + n)
    assert r <= RATIO_MAX


def _opposite_intact(case):
    """The opposite triangle and the padding still hold the sentinel bits."""
    import torch
    n, ldc, uplo = case["n"], case["ldc"], case["uplo"]
    i = torch.arange(ldc, device=case["C"][0].device)
    j = torch.arange(n, device=case["C"][0].device)
    # element (i, j) at [j*ldc + i]
    if uplo == "U":
        outside = i[None, :] > j[:, None]
    else:
        outside = (i[None, :] < j[:, None]) | (i[None, :] >= n)
    outside = outside | (i[None, :] >= n)
    for plane, s in ((case["C"][0], W.SENTINEL_HI), (case["C"][1], W.SENTINEL_LO)):
        want = int(np.array([s]).view(np.int64)[0])
        v = plane[: ldc * n].view(torch.int64).view(n, ldc)
        bad = (v != want) & outside
        assert not bool(bad.any()), "opposite triangle or padding changed"


@pytest.mark.parametrize("run", W.config2_runs(), ids=lambda r: f"{r[0]}{r[1]}-{r[2]}x{r[3]}")
@pytest.mark.parametrize("beta_zero", [True, False], ids=["beta0-nanC", "beta"])
def test_config2_rsyrk(h, run, beta_zero):
    uplo, trans, n, k = run
    case = W.syrk_case_device(W.BASE_SEED + 2 + n + k, uplo, trans, n, k, beta_zero=beta_zero)
    r = sampled_syrk_check(h, f"config2 {uplo}{trans} {n}x{k} beta0={beta_zero}", case,
                           seed=n + k)
    assert r <= RATIO_MAX
    _opposite_intact(case)
    log(f"PARITY config2 {uplo}{trans} {n}x{k} beta0={beta_zero} opposite-triangle intact")


@pytest.mark.parametrize("dist", ["uniform", "wide"])
def test_rgemm_8192_wide_and_uniform_accurate_form(h, dist):
    """Both input sets at n = 8192 with the plain form, and the accurate form
    on the wide set."""
    from paper_2109_13406_amd import binding as b
    case = W.gemm_case_device(W.BASE_SEED + 77, "N", "N", 8192, 8192, 8192, dist=dist)
    r = sampled_gemm_check(h, f"NN 8192 {dist} plain", case, seed=5)
    assert r <= RATIO_MAX
    if dist == "wide":
        case = W.gemm_case_device(W.BASE_SEED + 78, "T", "N", 2048, 2048, 2048, dist=dist)
        r = sampled_gemm_check(h, "TN 2048 wide accurate", case,
                               opts=dict(algo=b.MPDD_PLAIN_ACCURATE), seed=6)
        assert r <= RATIO_MAX

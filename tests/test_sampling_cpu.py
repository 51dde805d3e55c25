"""Host logic of the sampled parity checks: the compact sub-problem built from
sampled rows of op(A) and columns of op(B) gives, through the oracle, exactly
the sampled entries of the full oracle result (all nine Cgemm op forms)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import csub
from oracle.compare import bits


@pytest.mark.parametrize("op", W.COPS, ids=[a + b for a, b in W.COPS])
def test_csub_matches_full_oracle(op):
    m, n, k = 37, 29, 23
    c = W.cgemm_case(77, op[0], op[1], m, n, k)
    full = tuple(p.copy() for p in c["C"])
    assert oracle.cgemm(op[0], op[1], m, n, k, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"],
                        c["beta"], full, c["ldc"]) == 0
    rng = np.random.default_rng(1)
    I = np.sort(rng.choice(m, 7, replace=False))
    J = np.sort(rng.choice(n, 5, replace=False))
    s = csub(c, I, J)
    out = tuple(p.copy() for p in s["C"])
    assert oracle.cgemm(s["transa"], s["transb"], 7, 5, k, s["alpha"], s["A"], s["lda"], s["B"],
                        s["ldb"], s["beta"], out, s["ldc"]) == 0
    sel = (I[:, None] + J[None, :] * c["ldc"]).ravel(order="F")
    for p, q in zip(out, full):
        assert np.array_equal(bits(p), bits(q[sel]))

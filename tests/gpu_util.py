"""Helpers for the GPU parity tests: move seeded cases to the device, run the
HIP library through its C ABI, bring results back, compare with the oracle."""
import os
import sys

import numpy as np

import oracle
import workloads as W
from oracle.compare import bits, componentwise, ratio

RESULTS = os.environ.get("MPDD_PARITY_LOG", os.path.join(
    os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "_build", "parity.log"))


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


def op_abs(case, which):
    """|op(X)| of the hi plane as a dense numpy array: op(A) m x k (which
    "A"), op(B) k x n ("B"); for an Rsyrk case op(A) n x k and op(B) its
    transpose."""
    if "uplo" in case:
        n, k, ld, tr = case["n"], case["k"], case["lda"], case["trans"].upper()
        X = np.abs(case["A"][0][: ld * (k if tr == "N" else n)])
        X = X.reshape(-1, ld).T              # column-major storage rows x cols
        opa = X[:n, :k] if tr == "N" else X[:k, :n].T
        return opa if which == "A" else opa.T
    m, n, k = case["m"], case["n"], case["k"]
    if which == "A":
        ld, tr, rows, cols = case["lda"], case["transa"].upper(), m, k
        X = case["A"][0]
    else:
        ld, tr, rows, cols = case["ldb"], case["transb"].upper(), k, n
        X = case["B"][0]
    sr, sc = (rows, cols) if tr == "N" else (cols, rows)
    S = np.abs(X[: ld * sc]).reshape(sc, ld).T[:sr, :]
    return S if tr == "N" else S.T


def comp_full(G, O, case, m, n, ldc, tri=None):
    """Componentwise error (units of 2^-104) over the stored entries."""
    if min(m, n, case["k"]) == 0:
        return 0.0
    absab = op_abs(case, "A") @ op_abs(case, "B")
    i, j = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    sel = np.ones_like(i, dtype=bool) if tri is None else (i <= j if tri == "U" else i >= j)
    idx = (i + j * ldc)[sel]
    return componentwise(G[0][idx], G[1][idx], O[0][idx], O[1][idx], absab[sel],
                         case["alpha"], case["beta"], case["C"][0][idx])


def compare_full(name, G, O, m, n, k, ldc, tri=None, check_rest=True, C0=None, case=None):
    """Ratio over the stored entries; everything else bit-identical to C0.
    With the case's inputs, the componentwise error is logged too."""
    idx = entries_mask(m, n, ldc, tri)
    r = ratio(G[0][idx], G[1][idx], O[0][idx], O[1][idx], k)
    extra = ""
    if case is not None:
        extra = f" comp={comp_full(G, O, case, m, n, ldc, tri):.3g}"
    log(f"PARITY {name} ratio={r:.3g}{extra}")
    if check_rest and C0 is not None:
        rest = np.ones(G[0].shape[0], bool)
        rest[idx] = False
        assert np.array_equal(bits(G[0])[rest], bits(C0[0])[rest]), f"{name}: untouched region changed"
        assert np.array_equal(bits(G[1])[rest], bits(C0[1])[rest]), f"{name}: untouched region changed"
    return r


def sample_indices(m, n, count, seed, tri=None):
    return W.sample_indices(m, n, count, seed, tri)


# ---- full-size cases checked on sampled entries --------------------------------------

_gather_rows_opA = W.gather_op_rows
_gather_cols_opB = W.gather_op_cols


def sampled_oracle(transa, transb, k, alpha, A, lda, B, ldb, beta, cin, ii, jj,
                   with_abs=False):
    """Oracle values of the sampled entries (ii[t], jj[t]) of an update whose
    operands live on the device; cin = (hi, lo) host values of C at those
    entries before the update.  with_abs: also return (|op(A)| |op(B)|) at
    those entries (hi parts, binary64), the componentwise denominator."""
    s = len(ii)
    ta, tb = transa.upper() != "N", transb.upper() != "N"
    As = tuple(np.ascontiguousarray(_gather_rows_opA(x, lda, ta, ii, k)).ravel() for x in A)
    Bs = tuple(np.ascontiguousarray(_gather_cols_opB(x, ldb, tb, jj, k)).ravel() for x in B)
    Cs = (np.zeros(s * s), np.zeros(s * s))
    d = np.arange(s)
    Cs[0][d + d * s] = cin[0]
    Cs[1][d + d * s] = cin[1]
    ref = oracle.rgemm_entries("N", "N", s, s, k, alpha, As, s, Bs, k, beta, Cs, s, d, d)
    if not with_abs:
        return ref
    absab = np.einsum("lt,tl->t", np.abs(As[0].reshape(k, s)), np.abs(Bs[0].reshape(s, k)))
    return ref, absab


def gather(pair, flat_idx):
    import torch
    idx = torch.as_tensor(flat_idx, device=pair[0].device)
    return tuple(p[idx].cpu().numpy() for p in pair)


def sampled_gemm_check(h, name, case, opts=None, count=192, seed=0):
    """Run a device-resident Rgemm case and compare sampled entries with the
    oracle.  Returns the ratio over the sample."""
    from paper_2109_13406_amd import binding as b
    import torch
    m, n, k, ldc = case["m"], case["n"], case["k"], case["ldc"]
    ii, jj = sample_indices(m, n, count, seed)
    flat = ii + jj * ldc
    cin = gather(case["C"], flat)
    args = (case["transa"], case["transb"], m, n, k, case["alpha"], case["A"], case["lda"],
            case["B"], case["ldb"], case["beta"], case["C"], ldc)
    info = b.mpdd_Rgemm(h, *args) if opts is None else b.mpdd_Rgemm_ex(h, opts, *args)
    assert info == 0, info
    torch.cuda.synchronize()
    got = gather(case["C"], flat)
    ref, absab = sampled_oracle(case["transa"], case["transb"], k, case["alpha"], case["A"],
                                case["lda"], case["B"], case["ldb"], case["beta"], cin, ii, jj,
                                with_abs=True)
    r = ratio(got[0], got[1], ref[0], ref[1], k)
    c = componentwise(got[0], got[1], ref[0], ref[1], absab, case["alpha"], case["beta"], cin[0])
    log(f"PARITY {name} sampled({len(ii)}) ratio={r:.3g} comp={c:.3g}")
    return r


def sampled_syrk_check(h, name, case, opts=None, count=192, seed=0):
    from paper_2109_13406_amd import binding as b
    import torch
    n, k, ldc, uplo = case["n"], case["k"], case["ldc"], case["uplo"]
    ii, jj = sample_indices(n, n, count, seed, tri=uplo)
    flat = ii + jj * ldc
    cin = gather(case["C"], flat)
    if case["beta"] == (0.0, 0.0):
        cin = (np.zeros(len(ii)), np.zeros(len(ii)))
    args = (uplo, case["trans"], n, k, case["alpha"], case["A"], case["lda"], case["beta"],
            case["C"], ldc)
    info = b.mpdd_Rsyrk(h, *args) if opts is None else b.mpdd_Rsyrk_ex(h, opts, *args)
    assert info == 0, info
    torch.cuda.synchronize()
    got = gather(case["C"], flat)
    tr = case["trans"].upper()
    ref, absab = sampled_oracle(tr, "T" if tr == "N" else "N", k, case["alpha"], case["A"],
                                case["lda"], case["A"], case["lda"], case["beta"], cin, ii, jj,
                                with_abs=True)
    r = ratio(got[0], got[1], ref[0], ref[1], k)
    c = componentwise(got[0], got[1], ref[0], ref[1], absab, case["alpha"], case["beta"], cin[0])
    log(f"PARITY {name} sampled({len(ii)}) ratio={r:.3g} comp={c:.3g}")
    return r


def take(p, idx):
    """p[idx] as a numpy array, for a numpy plane or a device tensor."""
    if isinstance(p, np.ndarray):
        return p[idx]
    import torch
    return p[torch.from_numpy(np.ascontiguousarray(idx)).to(p.device)].cpu().numpy()


def csub(c, I, J):
    """The Cgemm case restricted to rows I of op(A) and columns J of op(B):
    compact operands with the same op flags, C = C[I, J].  Entry (r, s) of its
    result is entry (I[r], J[s]) of the full one, computed by the same steps.
    The planes may be numpy arrays or device tensors (gathered to the host)."""
    k, ta, tb = c["k"], c["transa"].upper(), c["transb"].upper()
    li, lj = len(I), len(J)
    ar = np.arange(k)
    A, B = [], []
    for p in c["A"]:
        if ta == "N":     # op(A) rows I = storage rows I: li x k
            A.append(take(p, (I[:, None] + ar[None, :] * c["lda"]).ravel(order="F")))
        else:             # storage columns I: k x li
            A.append(take(p, (ar[:, None] + I[None, :] * c["lda"]).ravel(order="F")))
    for p in c["B"]:
        if tb == "N":     # op(B) columns J = storage columns J: k x lj
            B.append(take(p, (ar[:, None] + J[None, :] * c["ldb"]).ravel(order="F")))
        else:             # storage rows J: lj x k
            B.append(take(p, (J[:, None] + ar[None, :] * c["ldb"]).ravel(order="F")))
    C = tuple(take(p, (I[:, None] + J[None, :] * c["ldc"]).ravel(order="F")) for p in c["C"])
    return dict(transa=ta, transb=tb, m=li, n=lj, k=k, alpha=c["alpha"], beta=c["beta"],
                A=tuple(A), lda=(li if ta == "N" else k), B=tuple(B), ldb=(k if tb == "N" else lj),
                C=C, ldc=li)

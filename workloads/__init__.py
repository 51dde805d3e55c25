"""Seeded synthetic inputs for the dd Rgemm / Rsyrk path.

This module is shared by the GPU tests, the benchmark and the oracle tests.
It holds no part of the method's arithmetic: it draws random binary64 numbers
with numpy and lays them out column-major; the only floating-point step is the
renormalisation of each generated (hi, lo) pair (hi <- fl(hi + lo),
lo <- the rounding error, exact because |lo| < |hi|), which is part of the
input recipe: values are normalised dd numbers.

Recipes (the dd matrices the manual's benchmarks feed to Rgemm / Rsyrk are
not published, so these stand in for them):

* "uniform": hi ~ U[-1, 1), lo = hi * 2^-53 * U[-1, 1), then renormalised.
* "wide":    hi = s * U[1, 2) * 2^e, e uniform integer in [-20, 20] drawn per
             entry, s a random sign; lo as for "uniform".

Seeds: numpy Generator(PCG64(seed)); the streams of one case are
SeedSequence(seed).spawn(5) in the order A, B, C, alpha, beta.
Padding rows (between the matrix's rows and its leading dimension) are filled
with a NaN sentinel so that reads or writes there are detectable.
"""
import math

import numpy as np

# Quiet-NaN sentinels with distinct payloads for the hi and lo planes.
SENTINEL_HI = np.array([0x7FF8DEAD00000001], dtype=np.uint64).view(np.float64)[0]
SENTINEL_LO = np.array([0x7FF8DEAD00000002], dtype=np.uint64).view(np.float64)[0]

BASE_SEED = 20260


def ld_padded(rows):
    """Leading dimension padded to the next multiple of 64, plus 3."""
    return 64 * max(1, math.ceil(rows / 64)) + 3


def streams(seed):
    """Five independent generators for A, B, C, alpha, beta."""
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(5)]


def _renorm(hi, lo):
    s = hi + lo
    e = lo - (s - hi)
    return s, e


def dd_values(rng, count, dist="uniform"):
    """`count` normalised dd numbers as (hi, lo) float64 arrays."""
    if dist == "uniform":
        hi = rng.uniform(-1.0, 1.0, count)
    elif dist == "wide":
        mant = rng.uniform(1.0, 2.0, count)
        e = rng.integers(-20, 21, count)
        sign = np.where(rng.integers(0, 2, count) == 0, -1.0, 1.0)
        hi = sign * np.ldexp(mant, e)
    elif dist == "int":
        hi = rng.integers(-8, 9, count).astype(np.float64)
        return hi, np.zeros(count)
    else:
        raise ValueError(dist)
    lo = hi * 2.0 ** -53 * rng.uniform(-1.0, 1.0, count)
    return _renorm(hi, lo)


def dd_scalar(rng, dist="uniform"):
    h, l = dd_values(rng, 1, dist)
    return float(h[0]), float(l[0])


def dd_matrix(rng, rows, cols, ld=None, dist="uniform", pad=True):
    """Column-major rows x cols dd matrix with leading dimension ld.

    Returns (hi, lo) flat float64 arrays of length ld*cols (at least 1).
    Entries (i, j) live at [i + j*ld]; padding rows hold the NaN sentinel."""
    ld = rows if ld is None else ld
    assert ld >= max(1, rows)
    size = max(1, ld * cols)
    hi = np.full(size, SENTINEL_HI if pad else 0.0)
    lo = np.full(size, SENTINEL_LO if pad else 0.0)
    if rows * cols:
        h, l = dd_values(rng, rows * cols, dist)
        v = hi[: ld * cols].reshape(cols, ld)
        v[:, :rows] = h.reshape(cols, rows)
        v = lo[: ld * cols].reshape(cols, ld)
        v[:, :rows] = l.reshape(cols, rows)
    return hi, lo


def fill_sentinel(hi, lo):
    hi[:] = SENTINEL_HI
    lo[:] = SENTINEL_LO


def view(flat, rows, cols, ld):
    """(rows, cols) numpy view of a column-major flat array (no copy)."""
    return flat[: ld * cols].reshape(cols, ld)[:, :rows].T if rows * cols else \
        np.zeros((rows, cols))


def gemm_case(seed, transa, transb, m, n, k, dist="uniform", padded=True, beta_zero=False,
              c_nan=False):
    """One seeded Rgemm case: dict with A, B, C (hi, lo), alpha, beta, lds."""
    ra, rb, rc, ral, rbe = streams(seed)
    nra = m if transa.upper() == "N" else k
    nca = k if transa.upper() == "N" else m
    nrb = k if transb.upper() == "N" else n
    ncb = n if transb.upper() == "N" else k
    lda = ld_padded(nra) if padded else max(1, nra)
    ldb = ld_padded(nrb) if padded else max(1, nrb)
    ldc = ld_padded(m) if padded else max(1, m)
    A = dd_matrix(ra, nra, nca, lda, dist)
    B = dd_matrix(rb, nrb, ncb, ldb, dist)
    C = dd_matrix(rc, m, n, ldc, dist)
    if c_nan:
        fill_sentinel(*C)
    alpha = dd_scalar(ral, "uniform")
    beta = (0.0, 0.0) if beta_zero else dd_scalar(rbe, "uniform")
    return dict(transa=transa, transb=transb, m=m, n=n, k=k, A=A, lda=lda, B=B, ldb=ldb,
                C=C, ldc=ldc, alpha=alpha, beta=beta)


def syrk_case(seed, uplo, trans, n, k, dist="uniform", padded=True, beta_zero=False):
    """One seeded Rsyrk case.  The triangle opposite to uplo (diagonal
    excluded) is filled with the NaN sentinel; with beta_zero the whole of C
    is the sentinel (it must not be read)."""
    ra, _, rc, ral, rbe = streams(seed)
    nra = n if trans.upper() == "N" else k
    nca = k if trans.upper() == "N" else n
    lda = ld_padded(nra) if padded else max(1, nra)
    ldc = ld_padded(n) if padded else max(1, n)
    A = dd_matrix(ra, nra, nca, lda, dist)
    C = dd_matrix(rc, n, n, ldc, dist)
    if n:
        i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        opp = (i > j) if uplo.upper() == "U" else (i < j)
        idx = (i + j * ldc)[opp]
        C[0][idx] = SENTINEL_HI
        C[1][idx] = SENTINEL_LO
    if beta_zero:
        fill_sentinel(*C)
    alpha = dd_scalar(ral, "uniform")
    beta = (0.0, 0.0) if beta_zero else dd_scalar(rbe, "uniform")
    return dict(uplo=uplo, trans=trans, n=n, k=k, A=A, lda=lda, C=C, ldc=ldc, alpha=alpha,
                beta=beta)


# ---- configurations ---------------------------------------------------------

SQUARE_SIZES = (1024, 2048, 4096, 8192)
OPS = ("NN", "NT", "TN", "TT")


def config1_runs():
    """Plain Rgemm runs: four op combinations x square sizes, plus the
    rectangular 4096x4096x256 and skinny 8192x64x8192 shapes."""
    runs = []
    for op in OPS:
        for s in SQUARE_SIZES:
            runs.append((op[0], op[1], s, s, s))
        runs.append((op[0], op[1], 4096, 4096, 256))
        runs.append((op[0], op[1], 8192, 64, 8192))
    return runs


def config2_runs():
    """Plain Rsyrk runs: uplo x trans x n x k."""
    return [(u, t, n, k) for u in "UL" for t in "NT" for n in (2048, 8192) for k in (512, 8192)]


# ---- served request stream -----------------------------------------------------

def request_stream(seed, count, rate, lo=32, hi=2048, gemm_frac=0.7):
    """Request descriptors for the serving workload.

    m, n, k = floor(exp(U[ln lo, ln(hi+1)))) (log-uniform integers in
    [lo, hi]); 70% Rgemm, 30% Rsyrk; flags uniform; Poisson arrivals (gaps
    exponential with mean 1/rate seconds).  Returns a list of dicts with
    'kind', flags, sizes, 'arrival' (seconds from start) and 'seed' (for the
    operands)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi + 1), (count, 3))))
    sizes = np.clip(sizes.astype(np.int64), lo, hi)
    kinds = rng.uniform(size=count) < gemm_frac
    flags = rng.integers(0, 2, (count, 2))
    gaps = rng.exponential(1.0 / rate, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for t in range(count):
        m, n, k = (int(x) for x in sizes[t])
        if kinds[t]:
            out.append(dict(kind="gemm", transa="NT"[flags[t, 0]], transb="NT"[flags[t, 1]],
                            m=m, n=n, k=k, arrival=float(arrivals[t]), seed=seed * 100003 + t))
        else:
            out.append(dict(kind="syrk", uplo="UL"[flags[t, 0]], trans="NT"[flags[t, 1]],
                            n=n, k=k, arrival=float(arrivals[t]), seed=seed * 100003 + t))
    return out

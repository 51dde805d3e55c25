"""Error metrics between a dd result and the oracle's (test infrastructure).

The tolerance unit is the dd machine epsilon 2^-104 (the manual's Table
"rlamch_dd", Rlamch('E') = 4.93038e-32).  For an update with inner dimension
k the normwise relative error over the checked entries is

    err = ||dC||_F / ||C_oracle||_F,   dC = (hi_g - hi_o) + (lo_g - lo_o),

and ratio = err / (k * 2^-104) (k >= 1).  A result passes when ratio <= 8.
When the oracle's norm is zero the difference must be exactly zero.

The componentwise report follows the manual's MPBLAS quality assurance
(section "Testing MPBLAS routines" compares every entry with a reference and
reports the largest error): for C_out = alpha op(A) op(B) + beta C_in,

    comp = max_ij |dC_ij| / (|alpha| (|op(A)| |op(B)|)_ij + |beta| |C_in,ij|)

in units of 2^-104.  The first-order error bound of a k-term dd dot product
puts the oracle itself within about (k + 4) of these units of the exact
result, so comp is reported beside the normwise ratio, not gated on its own.
"""
import numpy as np

EPS_DD = 2.0 ** -104
RATIO_MAX = 8.0


def diff(gh, gl, oh, ol):
    """Elementwise dd difference in binary64 (hi difference is exact for
    close values by Sterbenz)."""
    return (np.asarray(gh) - np.asarray(oh)) + (np.asarray(gl) - np.asarray(ol))


def ratio(gh, gl, oh, ol, k):
    """Normwise error ratio in units of k * 2^-104 (see module doc)."""
    d = diff(gh, gl, oh, ol)
    ref = np.asarray(oh, dtype=np.float64)
    if d.size == 0:
        return 0.0
    if not np.all(np.isfinite(d)):
        return float("inf")
    nref = np.linalg.norm(ref.ravel())
    nd = np.linalg.norm(d.ravel())
    if nref == 0.0:
        return 0.0 if nd == 0.0 else float("inf")
    return float(nd / nref / (max(int(k), 1) * EPS_DD))


def max_abs_ratio(gh, gl, oh, ol, k):
    """max |dC| / max |C_oracle| in units of k * 2^-104 (max-norm variant)."""
    d = np.abs(diff(gh, gl, oh, ol))
    ref = np.abs(np.asarray(oh))
    if d.size == 0:
        return 0.0
    m = ref.max()
    if m == 0.0:
        return 0.0 if d.max() == 0.0 else float("inf")
    return float(d.max() / m / (max(int(k), 1) * EPS_DD))


def componentwise(gh, gl, oh, ol, absab, alpha, beta, cin_hi):
    """max |dC_ij| / (|alpha| absab_ij + |beta| |cin_ij|) in units of 2^-104
    (see module doc); absab_ij = sum_l |a_il| |b_lj| of the hi parts (a
    binary64 estimate of the denominator is enough for a reported figure).
    alpha, beta: (hi, lo) pairs or numbers.  An entry whose denominator is 0
    must have dC = 0 (else the result is inf)."""
    d = np.abs(diff(gh, gl, oh, ol)).ravel()
    if d.size == 0:
        return 0.0
    if not np.all(np.isfinite(d)):
        return float("inf")
    a = abs(float(alpha[0] if np.ndim(alpha) else alpha))
    b = abs(float(beta[0] if np.ndim(beta) else beta))
    den = a * np.abs(np.asarray(absab, np.float64)).ravel()
    if b != 0.0:
        den = den + b * np.abs(np.asarray(cin_hi, np.float64)).ravel()
    zero = den == 0.0
    if np.any(d[zero] != 0.0):
        return float("inf")
    if np.all(zero):
        return 0.0
    return float((d[~zero] / den[~zero]).max() / EPS_DD)


def bits(a):
    """Raw 64-bit patterns (for bit-identity checks, NaN payloads included)."""
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)

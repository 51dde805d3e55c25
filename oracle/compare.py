"""Error metrics between a dd result and the oracle's (test infrastructure).

The tolerance unit is the dd machine epsilon 2^-104 (the manual's Table
"rlamch_dd", Rlamch('E') = 4.93038e-32).  For an update with inner dimension
k the normwise relative error over the checked entries is

    err = ||dC||_F / ||C_oracle||_F,   dC = (hi_g - hi_o) + (lo_g - lo_o),

and ratio = err / (k * 2^-104) (k >= 1).  A result passes when ratio <= 8.
When the oracle's norm is zero the difference must be exactly zero.
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


def bits(a):
    """Raw 64-bit patterns (for bit-identity checks, NaN payloads included)."""
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)

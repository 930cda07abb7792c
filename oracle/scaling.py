"""Power-of-two scaling before a half-precision LU (oracle; test infrastructure only).

Sec. 2.1.2 of the paper: rounding a higher-precision matrix to half precision
can overflow or underflow, so when the first LU attempt in half precision
produces Inf/NaN factors the factorization is retried after a two-sided
equilibration followed by a scalar that spreads the entries over the half
range (the squeezing method of Higham, Pranesh and Zounon, cited there).

Reading used here (the cited method is not restated in the paper):
  * R = diag(2^-e_i) with 2^(e_i - 1) <= max_j |a_ij| < 2^e_i  (row equilibration)
  * S = diag(2^-f_j), the same rule on the columns of R A
  * mu = 2^floor(log2(theta * xmax / max |R A S|)), theta = 2^-4, xmax the
    largest finite value of the factor format, leaving head-room for pivot growth.
All factors are powers of two, so R A S and mu R A S are exact in float64 and
A^{-1} = mu S (mu R A S)^{-1} R holds without rounding.  "Column scaling" is
the same with R = I.  Scaling is only used when u_f is fp16 (the format with
a narrow exponent range).
"""
import numpy as np

from . import fmt as F

THETA = 2.0 ** -4


def _pow2_equilibrator(maxabs):
    """2^-e with 2^(e-1) <= maxabs < 2^e; 1 where maxabs is zero or non-finite."""
    out = np.ones_like(maxabs)
    ok = np.isfinite(maxabs) & (maxabs > 0)
    _, e = np.frexp(maxabs[ok])          # maxabs = m 2^e, 0.5 <= m < 1
    out[ok] = np.ldexp(1.0, -e)
    return out


def compute(A, fmt_f, rows=True):
    """Return (R, S, mu) for A (float64).  ``rows=False`` gives column scaling only."""
    n = A.shape[0]
    absA = np.abs(A)
    if rows:
        R = _pow2_equilibrator(absA.max(axis=1))
    else:
        R = np.ones(n)
    RA = absA * R[:, None]
    S = _pow2_equilibrator(RA.max(axis=0))
    m = (RA * S[None, :]).max()
    if not (np.isfinite(m) and m > 0):
        return R, S, 1.0
    _, e = np.frexp(THETA * F.XMAX[fmt_f] / m)   # ratio = m' 2^e, 0.5 <= m' < 1
    return R, S, float(np.ldexp(1.0, int(e) - 1))


def apply(A, R, S, mu):
    """mu * R A S (exact: all factors are powers of two)."""
    return (mu * (R[:, None] * A)) * S[None, :]

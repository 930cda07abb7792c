"""Residuals and matrix-vector products in a named precision (oracle; test infrastructure only).

Alg. 4: "compute r_i = b - A x_i in precision u_r; scale r_i = r_i/||r_i||_inf;
store in precision u" (first line inside the loop, and Sec. 2.1.2 for the
scaling).  Alg. 2/3: the matrix-vector product with A inside GMRES is formed in
precision u^2 (GMRES-IR) or u (SGMRES-IR).

Readings used here:
  * u_r = fp64: r = b - A x with float64 arithmetic (library matrix-vector product).
  * u_r = dd:   r = b - A x in double-double (exact products via TwoProduct,
    double-double accumulation); r is returned as a (hi, lo) pair.
  * the scaled residual is fl_u(r_i / s) with s = ||r||_inf, the quotient
    formed in float64 (for a dd residual: fl_u(hi_i/s + lo_i/s)).
  * A v in precision p: p = fp32 uses A rounded to fp32 with the products
    summed in float64 and the result rounded to fp32; p = fp64 is the float64
    product; p = dd is the double-double product of the float64 A and v.
"""
import numpy as np

from . import dd
from .fmt import round_to

_CHUNK = 512


def dd_matvec(A, x, b=None):
    """(hi, lo) of b - A x (or of A x when b is None) in double-double."""
    A = np.asarray(A, dtype=np.float64)
    n, m = A.shape
    x = np.asarray(x, dtype=np.float64)
    if b is None:
        hi, lo = np.zeros(n), np.zeros(n)
        sign = 1.0
    else:
        hi, lo = np.array(b, dtype=np.float64, copy=True), np.zeros(n)
        sign = -1.0
    with np.errstate(all="ignore"):
        for j in range(m):
            ph, pl = dd.two_prod(A[:, j], np.full(n, x[j]))
            hi, lo = dd.add(hi, lo, sign * ph, sign * pl)
    return hi, lo


def residual(A, x, b, ur):
    """r = b - A x in precision ur ('fp64' -> float64 array, 'dd' -> (hi, lo))."""
    if ur == "fp64":
        with np.errstate(all="ignore"):
            return np.asarray(b, dtype=np.float64) - np.asarray(A, dtype=np.float64) @ np.asarray(x, dtype=np.float64)
    if ur == "dd":
        return dd_matvec(A, x, b)
    raise ValueError("residual precision must be fp64 or dd")


def rnorm_inf(r):
    """||r||_inf of a float64 vector or of a (hi, lo) pair (the float64 value of each entry)."""
    if isinstance(r, tuple):
        v = r[0] + r[1]
    else:
        v = r
    with np.errstate(invalid="ignore"):
        a = np.abs(v)
    if np.any(np.isnan(a)):
        return np.nan
    return float(a.max()) if a.size else 0.0


def scale_residual(r, s, u):
    """fl_u(r / s) (Alg. 4, residual scaling)."""
    with np.errstate(all="ignore"):
        if isinstance(r, tuple):
            q = r[0] / s + r[1] / s
        else:
            q = r / s
    return round_to(q, u)


def matvec(A, v, p, A_u=None):
    """A v in precision p.  Returns float64 values representable in p, or (hi, lo) for dd."""
    with np.errstate(all="ignore"):
        if p == "fp32":
            Au = A_u if A_u is not None else round_to(A, "fp32")
            return round_to(Au @ round_to(v, "fp32"), "fp32")
        if p == "fp64":
            return np.asarray(A) @ np.asarray(v, dtype=np.float64)
        if p == "dd":
            if isinstance(v, tuple):
                v = v[0]
            return dd_matvec(A, v)
    raise ValueError(p)

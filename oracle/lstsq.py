"""Least-squares MSIR (oracle; test infrastructure only).

Sec. 4 names the extension of the multistage approach to least squares problems
min ||b - A x||_2 (A m x n, m >= n, full column rank) as future work, to be built
from the error bounds for least squares refinement and the three-precision schemes
for least squares it cites.  The classical way to refine a least squares solution is
refinement on the augmented system

    [ alpha I   A ] [ y ]   [ b ]
    [ A^T       0 ] [ x ] = [ 0 ],        r = b - A x = alpha y,

whose second block row states the normal equations A^T r = 0.  This module takes
that route with Alg. 4 unchanged: the multistage controller (oracle.msir.msir) runs on
the (m + n) x (m + n) augmented matrix, so the LU in u_f, the SIR / SGMRES-IR /
GMRES-IR switches and the precision escalation all apply to it as they do to a square
system.  Readings (no passage fixes them):

  * alpha is a power of two, so that alpha I and r = alpha y are exact.  Default:
    the largest power of two not above max |a_ij| (the two blocks then have entries of
    the same magnitude for the LU's pivoting).  The augmented matrix is best
    conditioned near alpha = sigma_min(A) / sqrt(2); a caller who knows sigma_min may
    pass such an alpha.
  * x and r come from the refined augmented solution; the history, the number of
    factorizations and the convergence test are those of the augmented system.
"""
import math

import numpy as np

from . import msir as OM


def alpha_default(A):
    """Largest power of two <= max |a_ij| (1 for A = 0)."""
    amax = float(np.max(np.abs(A))) if A.size else 0.0
    if not (amax > 0.0) or not math.isfinite(amax):
        return 1.0
    m, e = math.frexp(amax)          # amax = m 2^e, 0.5 <= m < 1
    return math.ldexp(1.0, e - 1)


def augment(A, b, alpha):
    """The augmented matrix [[alpha I, A], [A^T, 0]] and right-hand side [b; 0] (exact)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    N = m + n
    K = np.zeros((N, N))
    K[:m, :m] = alpha * np.eye(m)
    K[:m, m:] = A
    K[m:, :m] = A.T
    f = np.zeros(N)
    f[:m] = b
    return np.asfortranarray(K), f


def lstsq(A, b, params=OM.Params(), alpha=None):
    """Alg. 4 on the augmented system.  Returns (x, r, alpha, oracle.msir.Result)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("least squares needs m >= n")
    a = alpha_default(A) if alpha is None else float(alpha)
    K, f = augment(A, b, a)
    res = OM.msir(K, f, params)
    y = res.x[:m]
    x = res.x[m:].copy()
    r = a * y
    return x, r, a, res

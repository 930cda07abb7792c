"""Triangular solves with the stored LU factors (oracle; test infrastructure only).

Used by the initial solve and by SIR (Alg. 4: "compute d = U^{-1}(L^{-1} r) in
precision u_f", Table 1 "tri. solves") and inside GMRES as the left
preconditioner M^{-1} = U^{-1} L^{-1} P (Alg. 2 and 3), where it is applied in
precision u (SGMRES-IR) or u^2 (GMRES-IR).

Reading used here.  Plain row-by-row substitution.  ``comp`` is the format
every computed solution component is rounded to (u_f for the u_f-precision
solve; the operator precision p in GMRES).  Each inner product
sum_k T_rk y_k is accumulated in float64 (double-double when comp == "dd"),
which is at least as wide as the accumulator any of the formats needs.  The
backward sweep multiplies by the float64 reciprocal of the pivot (double-double
division when comp == "dd").  When the factorization was scaled
(mu R A S = L U) the solve returns mu S U^{-1} L^{-1} P R t, all scalings being
exact powers of two.
"""
import numpy as np

from . import dd
from .fmt import round_to


def _round_scalar(v, comp):
    if comp == "fp64":
        return v
    if comp == "fp32":
        return float(np.float32(v))
    if comp == "fp16":
        return float(np.float16(v))
    return float(round_to(np.array([v]), comp)[0])


def permute(t, piv):
    """P t for LAPACK-style interchanges (t is copied)."""
    t = np.array(t, dtype=np.float64, copy=True)
    for j, k in enumerate(piv):
        if k != j:
            t[j], t[k] = t[k], t[j]
    return t


def lu_solve(W, piv, t, comp, scal=None):
    """y = mu S U^{-1} L^{-1} P R t with every component rounded to ``comp``.

    ``t`` is a float64 vector (for comp == "dd" it may be a (hi, lo) pair).
    Returns float64 (or a (hi, lo) pair for comp == "dd").
    """
    if comp == "dd":
        return _lu_solve_dd(W, piv, t, scal)
    n = W.shape[0]
    t = np.asarray(t, dtype=np.float64)
    if scal is not None:
        R, S, mu = scal
        t = R * t
    acc = permute(t, piv)
    with np.errstate(all="ignore"):
        acc = round_to(acc, comp)
        y = np.empty(n)
        # forward: unit lower triangular L (strict lower part of W)
        for c in range(n):
            yc = _round_scalar(acc[c], comp)
            y[c] = yc
            if c + 1 < n:
                acc[c + 1:] -= W[c + 1:, c] * yc
        # backward: U (upper part of W including the diagonal)
        inv = 1.0 / np.diag(W)
        acc = y
        x = np.empty(n)
        for c in range(n - 1, -1, -1):
            xc = _round_scalar(acc[c] * inv[c], comp)
            x[c] = xc
            if c > 0:
                acc[:c] -= W[:c, c] * xc
        if scal is not None:
            x = mu * (S * x)
    return x


def _lu_solve_dd(W, piv, t, scal):
    n = W.shape[0]
    if isinstance(t, tuple):
        th, tl = (np.asarray(a, dtype=np.float64) for a in t)
    else:
        th, tl = np.asarray(t, dtype=np.float64), np.zeros(n)
    if scal is not None:
        R, S, mu = scal
        th, tl = R * th, R * tl
    ah, al = permute(th, piv), permute(tl, piv)
    with np.errstate(all="ignore"):
        for c in range(n):
            if c + 1 < n:
                ph, pl = dd.mul_d(np.full(n - c - 1, ah[c]), np.full(n - c - 1, al[c]), W[c + 1:, c])
                ah[c + 1:], al[c + 1:] = dd.add(ah[c + 1:], al[c + 1:], -ph, -pl)
        diag = np.diag(W).copy()
        for c in range(n - 1, -1, -1):
            qh, ql = dd.div(np.array([ah[c]]), np.array([al[c]]), np.array([diag[c]]), np.zeros(1))
            ah[c], al[c] = qh[0], ql[0]
            if c > 0:
                ph, pl = dd.mul_d(np.full(c, ah[c]), np.full(c, al[c]), W[:c, c])
                ah[:c], al[:c] = dd.add(ah[:c], al[:c], -ph, -pl)
        if scal is not None:
            ah, al = mu * (S * ah), mu * (S * al)
    return ah, al

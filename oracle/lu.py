"""LU factorization with partial pivoting, factors stored in u_f (oracle; test infrastructure only).

Alg. 4 (first line) and Alg. 1-3: "compute the LU factorization A = LU in
precision u_f" by Gaussian elimination with partial pivoting (Sec. 1).

Reading used here (the paper simulated u_f with the chop library, rounding
every scalar operation; hardware with matrix cores instead computes in a wider
format and stores in u_f).  The factorization is the right-looking blocked
elimination with block width ``nb``, all factor entries being rounded to u_f
whenever they are written back to the matrix:

  for each column block J = [j0, j0 + nb):
    1. panel: the columns of J below row j0 are taken into the arithmetic format
       (fp32 for u_f in {fp16, bf16, fp32}; fp64 for u_f = fp64).  For each
       column c: the pivot is the first row of largest magnitude (NaN never
       wins); rows are interchanged across the whole matrix; the multipliers are
       the column times the rounded reciprocal of the pivot; the rest of the
       panel gets a rank-1 update with fused multiply-adds.  A zero pivot
       column records info = c + 1 and is left unscaled (as LAPACK does).
       The panel is then rounded to u_f.
    2. U12 = L11^{-1} A12 by forward substitution with fused multiply-adds in
       the arithmetic format (row c uses rows 0..c-1 in increasing order),
       then rounded to u_f.
    3. A22 <- fl_f(fl_arith(A22 - L21 U12)), the product being formed from the
       stored u_f values: in fp32 arithmetic a chain of single-rounded fp32 fused
       multiply-adds in increasing k (the default; trailing="exact" rounds the
       exact float64 product once instead, a comparison model only); in float64
       arithmetic the products summed in increasing k, then subtracted.

For u_f = fp64 the panel and triangular updates use separately rounded
float64 multiply and subtract.  From order NATIVE_MIN_N on (the trailing chain
or float64 arithmetic) the same steps run as plain C loops (oracle/native/dm_lu.c,
pinned bit for bit against these Python loops) when that library is built.  ``piv`` uses LAPACK's convention (0-based):
at step j rows j and piv[j] were interchanged.
"""
import numpy as np

from . import native as _native
from .fmt import fma32, round_to

NATIVE_MIN_N = 384


def nb_auto(n, fmt_f):
    """Default panel width: the panel of the device kernels lives in registers of one
    compute unit (1024 threads, at most 64 fp32 or 32 fp64 values per thread), so the
    width is 64 / ceil(n / 1024) rounded down to a power of two, halved for fp64."""
    R = -(-n // 1024)
    nb = 64 if R <= 1 else 32 if R <= 2 else 16 if R <= 4 else 8 if R <= 8 else 4
    return nb // 2 if fmt_f == "fp64" else nb


def arith_format(fmt_f):
    return "fp64" if fmt_f == "fp64" else "fp32"


def _fma(wa):
    if wa == "fp32":
        return fma32
    return lambda a, b, c: c + a * b          # float64, two roundings


def getrf(A, fmt_f, nb=None, trailing="fma32", native=None):
    """Factor A (float64, values representable in fmt_f).

    Returns (W, piv, info): W holds the unit lower triangle of L below the
    diagonal and U on and above it, all entries representable in fmt_f.
    native: True / False forces the C or the Python loops; None chooses C from
    order NATIVE_MIN_N on when it is built (the two agree bit for bit).
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if nb is None:
        nb = nb_auto(n, fmt_f)
    same_steps = trailing == "fma32" or arith_format(fmt_f) == "fp64"
    if native is None:
        native = same_steps and n >= NATIVE_MIN_N and _native.available()
    if native:
        if not same_steps:
            raise ValueError("the C loops implement the fma32 trailing chain (and float64 arithmetic) only")
        return _native.getrf(A, fmt_f, nb)
    W = np.array(A, dtype=np.float64, order="F", copy=True)
    piv = np.arange(n, dtype=np.int64)
    info = 0
    wa = arith_format(fmt_f)
    fma = _fma(wa)

    def rnd(x):
        return round_to(x, wa)

    for j0 in range(0, n, nb):
        jb = min(nb, n - j0)
        P = W[j0:, j0:j0 + jb].copy()
        for c in range(jb):
            col = np.abs(P[c:, c])
            valid = ~np.isnan(col)
            if valid.any():
                m = col[valid].max()
                idx = int(np.flatnonzero(valid & (col == m))[0])
            else:
                m = np.nan
                idx = 0
            p = c + idx
            piv[j0 + c] = j0 + p
            if p != c:
                P[[c, p], :] = P[[p, c], :]
                W[[j0 + c, j0 + p], :j0] = W[[j0 + p, j0 + c], :j0]
                W[[j0 + c, j0 + p], j0 + jb:] = W[[j0 + p, j0 + c], j0 + jb:]
            if not (m > 0):
                if info == 0:
                    info = j0 + c + 1
                continue
            with np.errstate(all="ignore"):
                rcp = rnd(1.0 / P[c, c])
                P[c + 1:, c] = rnd(P[c + 1:, c] * rcp)
                if c + 1 < jb:
                    P[c + 1:, c + 1:] = fma(-P[c + 1:, c:c + 1], P[c:c + 1, c + 1:], P[c + 1:, c + 1:])
        W[j0:, j0:j0 + jb] = round_to(P, fmt_f)
        if j0 + jb < n:
            L11 = W[j0:j0 + jb, j0:j0 + jb]
            U12 = W[j0:j0 + jb, j0 + jb:].copy()
            with np.errstate(all="ignore"):
                for c in range(1, jb):
                    for k in range(c):
                        U12[c] = fma(-L11[c, k], U12[k], U12[c])
            U12 = round_to(U12, fmt_f)
            W[j0:j0 + jb, j0 + jb:] = U12
            L21 = W[j0 + jb:, j0:j0 + jb]
            with np.errstate(all="ignore"):
                if trailing == "fma32" and wa == "fp32":
                    acc = W[j0 + jb:, j0 + jb:].copy()
                    for k in range(jb):
                        acc = fma32(-L21[:, k:k + 1], U12[k:k + 1, :], acc)
                    W[j0 + jb:, j0 + jb:] = round_to(acc, fmt_f)
                elif wa == "fp64":
                    acc = np.zeros_like(W[j0 + jb:, j0 + jb:])
                    for k in range(jb):
                        acc = acc + L21[:, k:k + 1] * U12[k:k + 1, :]
                    W[j0 + jb:, j0 + jb:] = W[j0 + jb:, j0 + jb:] - acc
                else:
                    W[j0 + jb:, j0 + jb:] = round_to(rnd(W[j0 + jb:, j0 + jb:] - L21 @ U12), fmt_f)
    return W, piv, info


def unpack(W):
    """(L, U) as dense float64 matrices."""
    L = np.tril(W, -1) + np.eye(W.shape[0])
    U = np.triu(W)
    return L, U


def perm_from_piv(piv):
    """Row permutation p with (P A)[i] = A[p[i]] for LAPACK-style interchanges."""
    n = len(piv)
    p = np.arange(n)
    for j in range(n):
        k = piv[j]
        if k != j:
            p[j], p[k] = p[k], p[j]
    return p

"""Left-preconditioned GMRES for the correction equation (oracle; test infrastructure only).

Alg. 2 (GMRES-IR) and Alg. 3 (SGMRES-IR): solve U^{-1} L^{-1} A d = U^{-1} L^{-1} r
by GMRES in working precision u, the preconditioned matrix being applied in
precision p = u^2 (GMRES-IR) or p = u (SGMRES-IR).  Convergence: the relative
preconditioned residual drops below tau (Sec. 2, motivating example); the
number of iterations is limited by k_max (Sec. 2.1.1, fourth criterion).

Readings used here (the paper does not spell these out): initial guess 0;
modified Gram-Schmidt Arnoldi; Givens rotations on the Hessenberg matrix;
inner products, norms, the Hessenberg matrix and the small least-squares
problem in float64; every vector that GMRES stores (Krylov basis, the
preconditioned residual, the correction) rounded to u; the update
w <- w - h v_i formed with separately rounded float64 multiply and subtract
before rounding to u.  The iteration stops when |g_{j+1}| <= tau * beta0
(beta0 the 2-norm of the first preconditioned residual of this call), when
the Arnoldi vector vanishes, or after k_cap = ceil(k_max) iterations.  With
restart length m > 0 the basis is discarded every m iterations: the
correction so far is accumulated in float64 and the preconditioned residual is
updated as fl_u(c - fl_u(M^{-1} A delta)) with delta the cycle's correction
rounded to u.
"""
import math

import numpy as np

from .fmt import round_to
from .ops import matvec
from .solve import lu_solve


def _to_u(y, u):
    if isinstance(y, tuple):
        with np.errstate(all="ignore"):
            y = y[0] + y[1]
    return round_to(y, u)


def precond_apply(A, W, piv, scal, v, p, u, A_u=None):
    """fl_u(M^{-1} A v) with A v and the triangular solves in precision p."""
    return _to_u(lu_solve(W, piv, matvec(A, v, p, A_u=A_u), p, scal), u)


def gmres(A, W, piv, scal, rhat, u, p, tau, k_max, restart=0, A_u=None, trace=None):
    """Return (d, k): d (float64 array of u values) and the iteration count k."""
    n = A.shape[0]
    k_cap = int(math.ceil(k_max))
    c = _to_u(lu_solve(W, piv, rhat, p, scal), u)
    with np.errstate(all="ignore"):
        beta0 = float(np.sqrt(np.dot(c, c)))
    if not np.isfinite(beta0):
        return np.full(n, np.nan), 0
    d = np.zeros(n)
    if beta0 == 0.0:
        return d, 0
    k = 0
    resid = c
    while True:
        with np.errstate(all="ignore"):
            beta = float(np.sqrt(np.dot(resid, resid)))
        m = restart if restart > 0 else k_cap
        m = min(m, k_cap - k)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        with np.errstate(all="ignore"):
            V[0] = round_to(resid / beta, u)
        j = 0
        stop = False
        while j < m:
            w = precond_apply(A, W, piv, scal, V[j], p, u, A_u)
            k += 1
            with np.errstate(all="ignore"):
                for i in range(j + 1):
                    h = float(np.dot(V[i], w))
                    H[i, j] = h
                    w = round_to(w - h * V[i], u)
                hn = float(np.sqrt(np.dot(w, w)))
                H[j + 1, j] = hn
                for i in range(j):
                    a, b = H[i, j], H[i + 1, j]
                    H[i, j] = cs[i] * a + sn[i] * b
                    H[i + 1, j] = -sn[i] * a + cs[i] * b
                a, b = H[j, j], H[j + 1, j]
                r = math.hypot(a, b)
                if r == 0.0:
                    cs[j], sn[j] = 1.0, 0.0
                else:
                    cs[j], sn[j] = a / r, b / r
                H[j, j] = r
                H[j + 1, j] = 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
            j += 1
            if trace is not None:
                trace.append(abs(g[j]) / beta0)
            if not np.isfinite(g[j]) or abs(g[j]) <= tau * beta0 or hn == 0.0:
                stop = True
                break
            with np.errstate(all="ignore"):
                V[j] = round_to(w / hn, u)
        # y = R^{-1} g (upper triangular, float64), delta = fl_u(V y)
        y = np.zeros(j)
        with np.errstate(all="ignore"):
            for i in range(j - 1, -1, -1):
                y[i] = (g[i] - np.dot(H[i, i + 1:j], y[i + 1:j])) / H[i, i]
            delta = round_to(V[:j].T @ y, u)
            d = d + delta
        if stop or k >= k_cap:
            break
        with np.errstate(all="ignore"):
            resid = round_to(resid - precond_apply(A, W, piv, scal, delta, p, u, A_u), u)
    return round_to(d, u), k

"""Error measures of Sec. 2 (oracle; test infrastructure only).

ferr = ||x_hat - x||_inf / ||x||_inf; normwise relative backward error
nbe = ||b - A x_hat|| / (||A|| ||x_hat|| + ||b||) (the inf-norm is used); and the
componentwise relative backward error cbe = max_i |b - A x_hat|_i / (|A| |x_hat| + |b|)_i.
The residual is formed in double-double so that the measure itself adds no
error at the float64 level.
"""
import numpy as np

from .ops import dd_matvec


def ferr(xh, x):
    return float(np.abs(xh - x).max() / np.abs(x).max())


def nbe(A, xh, b):
    hi, lo = dd_matvec(A, xh, b)
    r = np.abs(hi + lo).max()
    return float(r / (np.abs(A).sum(axis=1).max() * np.abs(xh).max() + np.abs(b).max()))


def cbe(A, xh, b):
    hi, lo = dd_matvec(A, xh, b)
    num = np.abs(hi + lo)
    den = np.abs(A) @ np.abs(xh) + np.abs(b)
    with np.errstate(all="ignore"):
        q = np.where(den > 0, num / den, np.where(num > 0, np.inf, 0.0))
    return float(q.max())

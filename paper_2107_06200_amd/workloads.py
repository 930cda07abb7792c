"""Seeded synthetic inputs shaped like the paper's random dense test problems.

Sec. 3.1 of the paper tests MATLAB ``gallery('randsvd', n, kappa, mode)``
matrices: mode 2 has one singular value 1/kappa and the others 1; mode 3 has
geometrically distributed singular values from 1 to 1/kappa.  The MATLAB
matrices cannot be regenerated here, so this module builds the same families
from numpy's PCG64 stream: A = U diag(sigma) V^T with U, V Haar-distributed
orthogonal matrices (QR of a standard Gaussian matrix with the signs of R's
diagonal moved into Q), x_true ~ N(0, 1) and b = A x_true in float64.

This module holds only input construction (no part of the solver's arithmetic)
and is the one piece of code shared by the tests, the benchmark and callers
of the CPU oracle.  Nothing in it imports the HIP library.
"""
import math

import numpy as np


def rng_for(config_id, index=0):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(config_id), int(index)])))


def haar_orthogonal(rng, n):
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))[None, :]


def singular_values(n, kappa, mode):
    if mode == 2:
        s = np.ones(n)
        s[-1] = 1.0 / kappa
        return s
    if mode == 3:
        if n == 1:
            return np.ones(1)
        return kappa ** (-np.arange(n) / (n - 1.0))
    raise ValueError("mode must be 2 or 3")


def randsvd(n, kappa, mode, rng, nrhs=0):
    """(A, x_true, b) in float64, A in Fortran (column-major) order."""
    U = haar_orthogonal(rng, n)
    V = haar_orthogonal(rng, n)
    s = singular_values(n, kappa, mode)
    A = np.asfortranarray((U * s[None, :]) @ V.T)
    if nrhs:
        x = rng.standard_normal((n, nrhs))
    else:
        x = rng.standard_normal(n)
    b = A @ x
    return A, x, b


def ls_system(m, n, kappa, mode, rng, rnorm=1e-2):
    """Least-squares problem (A, x_true, b, r_true): A = U diag(s) V^T with U m x n
    orthonormal columns (the first n columns of a Haar orthogonal matrix), s the
    randsvd singular values, x_true ~ N(0, 1); r_true orthogonal to range(A) (the
    remaining columns of the same orthogonal matrix), scaled to rnorm ||A x_true||_2;
    b = A x_true + r_true.  The least-squares solution is x_true and its residual
    r_true (up to rounding in forming b)."""
    Q = haar_orthogonal(rng, m)
    V = haar_orthogonal(rng, n)
    s = singular_values(n, kappa, mode)
    A = np.asfortranarray((Q[:, :n] * s[None, :]) @ V.T)
    x = rng.standard_normal(n)
    Ax = A @ x
    if m > n:
        c = rng.standard_normal(m - n)
        r = Q[:, n:] @ c
        r *= rnorm * np.linalg.norm(Ax) / np.linalg.norm(r)
    else:
        r = np.zeros(m)
    return A, x, Ax + r, r


def kappa_inf(A):
    """Infinity-norm condition number (computed with a float64 inverse)."""
    return float(np.abs(A).sum(axis=1).max() * np.abs(np.linalg.inv(A)).sum(axis=1).max())


# The five workloads of the benchmark table.  Each entry gives the input recipe and
# the solver parameters named with the paper's symbols.
CONFIGS = {
    1: dict(name="sir_n100", n=100, kappa=1e2, mode=3,
            params=dict(uf="fp16", u="fp32", ur="fp64", ux="fp64", i_max=10, tau=1e-6,
                        rho_thresh=0.5, k_max=10, restart=0, scaling="auto")),
    2: dict(name="msir_n4096_k1e6_mode3", n=4096, kappa=1e6, mode=3,
            params=dict(uf="fp16", u="fp32", ur="fp64", ux="fp64", i_max=10, tau=1e-4,
                        rho_thresh=0.5, k_max=None, restart=50, scaling="cols")),
    3: dict(name="gmresir_n8192_k1e10_mode2", n=8192, kappa=1e10, mode=2,
            params=dict(uf="fp16", u="fp64", ur="dd", ux="fp64", i_max=10, tau=1e-10,
                        rho_thresh=0.5, k_max=None, restart=0, scaling="auto")),
}


def config_system(cid, index=0, n=None):
    """Inputs of one configured single system (n may be overridden for scaled-down tests)."""
    c = CONFIGS[cid]
    nn = c["n"] if n is None else n
    return randsvd(nn, c["kappa"], c["mode"], rng_for(cid, index))


def batched_meta(count=512, nmin=64, nmax=1024, seed=4):
    """Orders and conditioning of the uneven batch: n log-uniform in [nmin, nmax],
    log10 kappa ~ U[1, 8], modes 2 (even index) and 3 (odd index)."""
    meta = rng_for(seed, 10 ** 6)
    out = []
    for i in range(count):
        n = int(round(math.exp(meta.uniform(math.log(nmin), math.log(nmax)))))
        kappa = 10.0 ** meta.uniform(1.0, 8.0)
        out.append(dict(index=i, n=n, kappa=kappa, mode=2 if i % 2 == 0 else 3))
    return out


def batched_system(m, seed=4):
    """(A, x_true, b) of one entry of batched_meta."""
    return randsvd(m["n"], m["kappa"], m["mode"], rng_for(seed, m["index"]))


def batched_systems(count=512, nmin=64, nmax=1024, seed=4):
    """Uneven batch: n log-uniform in [nmin, nmax], log10 kappa ~ U[1, 8], modes 2/3 alternating."""
    out = []
    for m in batched_meta(count, nmin, nmax, seed):
        A, x, b = batched_system(m, seed)
        out.append(dict(m, A=A, x=x, b=b))
    return out


# Solver parameters of the uneven batch (fp16 factors, fp32 working precision, fp64
# residual, GMRES tolerance 1e-6, k_max = 0.1 n by default).
BATCHED_PARAMS = dict(uf="fp16", u="fp32", ur="fp64", ux="fp64", i_max=10, tau=1e-6, rho_thresh=0.5,
                      k_max=None, restart=0, scaling="auto")


def serving_requests(count=2000, sizes=(256, 512, 1024, 2048, 4096), seed=5, rate=1.0):
    """Request descriptors: arrival time (Poisson, ``rate`` per second), n, kappa, mode, nrhs.

    Matrices are built lazily with ``request_system`` so a long request stream
    does not have to be materialized at once.
    """
    meta = rng_for(seed, 10 ** 6)
    t = 0.0
    reqs = []
    for i in range(count):
        t += meta.exponential(1.0 / rate)
        reqs.append(dict(id=i, t=t, n=int(sizes[meta.integers(len(sizes))]),
                         kappa=10.0 ** meta.uniform(2.0, 8.0), mode=2 if i % 2 == 0 else 3,
                         nrhs=int(meta.integers(1, 17))))
    return reqs


def request_system(req, seed=5):
    return randsvd(req["n"], req["kappa"], req["mode"], rng_for(seed, req["id"]), nrhs=req["nrhs"])


def sparse_system(n, per_row, scale, rng):
    """Synthetic sparse system standing in for the paper's sparse test matrices.

    Each row holds its diagonal and per_row - 1 off-diagonal entries at random
    distinct columns (N(0, 1) values); the diagonal is (1.5 + U[0, 1]) sqrt(per_row - 1),
    which keeps the pattern matrix reasonably conditioned.  Rows and columns are then
    scaled by scale**U[0, 1] (independent per row and per column), which spreads the
    magnitudes and raises the condition number up to about scale^2 times.
    Returns (rowptr int32 n+1, colind int32 nnz, vals float64 nnz, A dense float64,
    x_true, b = A x_true).
    """
    k = per_row - 1
    cols = np.empty((n, per_row), dtype=np.int64)
    vals = rng.standard_normal((n, per_row))
    for i in range(n):
        c = rng.choice(n - 1, size=k, replace=False)
        c[c >= i] += 1
        cols[i, 0] = i
        cols[i, 1:] = c
        vals[i, 0] = (1.5 + rng.random()) * math.sqrt(max(k, 1))
    order = np.argsort(cols, axis=1)
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    dr = scale ** rng.random(n)
    dc = scale ** rng.random(n)
    vals = vals * dr[:, None] * dc[cols]
    rowptr = (np.arange(n + 1) * per_row).astype(np.int32)
    colind = cols.reshape(-1).astype(np.int32)
    v = vals.reshape(-1).astype(np.float64)
    A = np.zeros((n, n))
    A[np.repeat(np.arange(n), per_row), colind] = v
    x = rng.standard_normal(n)
    b = A @ x
    return rowptr, colind, v, A, x, b

"""Pins for double-double arithmetic, residuals and the oracle's GMRES.

Double-double: error-free transformations checked against exact rational sums
and products; the residual b - A x in double-double against an exact rational
residual.  GMRES: with an exact preconditioner (float64 LU of a
well-conditioned matrix) the preconditioned operator is the identity up to
rounding, so GMRES must converge in one iteration to A^{-1} r; with A = the
identity and a perturbed "LU" the iterate must match numpy's least-squares
solution of the Hessenberg problem; restarting with a length beyond the
iteration count must not change anything.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import dd, fmt as F, gmres as G, lu as LU, ops


def test_two_sum_two_prod_exact():
    rng = np.random.default_rng(0)
    a = rng.standard_normal(500) * np.exp2(rng.integers(-40, 40, 500))
    b = rng.standard_normal(500) * np.exp2(rng.integers(-40, 40, 500))
    s, e = dd.two_sum(a, b)
    p, f = dd.two_prod(a, b)
    for i in range(500):
        assert Fraction(s[i]) + Fraction(e[i]) == Fraction(a[i]) + Fraction(b[i])
        assert Fraction(p[i]) + Fraction(f[i]) == Fraction(a[i]) * Fraction(b[i])


def test_dd_residual_against_rationals():
    rng = np.random.default_rng(1)
    n = 12
    A = rng.standard_normal((n, n))
    x = rng.standard_normal(n)
    b = A @ x + rng.standard_normal(n) * 1e-14
    hi, lo = ops.residual(A, x, b, "dd")
    for i in range(n):
        exact = Fraction(b[i]) - sum(Fraction(A[i, j]) * Fraction(x[j]) for j in range(n))
        scale = sum(abs(Fraction(A[i, j]) * Fraction(x[j])) for j in range(n)) + abs(Fraction(b[i]))
        assert abs(Fraction(hi[i]) + Fraction(lo[i]) - exact) <= scale * n * Fraction(2) ** -104


def test_scaled_residual_definition():
    r = np.array([3.0, -1.5, 0.25])
    s = ops.rnorm_inf(r)
    assert s == 3.0
    np.testing.assert_array_equal(ops.scale_residual(r, s, "fp32"), F.round_to(r / 3.0, "fp32"))
    hi = np.array([1.0, -3.0]); lo = np.array([2.0 ** -60, 2.0 ** -58])
    q = ops.scale_residual((hi, lo), 3.0, "fp64")
    np.testing.assert_array_equal(q, hi / 3.0 + lo / 3.0)


@pytest.mark.parametrize("u,p", [("fp32", "fp32"), ("fp32", "fp64"), ("fp64", "fp64"), ("fp64", "dd")])
def test_gmres_exact_preconditioner_one_iteration(u, p):
    n = 24
    rng = np.random.default_rng(2)
    A = rng.standard_normal((n, n)) + 6 * np.eye(n)
    W, piv, _ = LU.getrf(A, "fp64", 8)
    r = F.round_to(rng.standard_normal(n), u)
    d, k = G.gmres(A, W, piv, None, r, u, p, tau=1e-6 if u == "fp32" else 1e-12, k_max=10)
    assert k <= 2
    want = np.linalg.solve(A, r)
    assert np.abs(d - want).max() <= 50 * F.u(u) * np.abs(want).max()


def test_gmres_lstsq_and_arnoldi():
    # a poor preconditioner (fp16 LU of A + noise) forces several iterations;
    # the final correction must equal V y with y the least-squares solution of
    # min ||beta e1 - H y|| and the residual must fall below tau.
    n = 40
    rng = np.random.default_rng(3)
    A = rng.standard_normal((n, n)) + 2 * np.eye(n)
    Af = F.round_to(A + 0.05 * rng.standard_normal((n, n)), "fp16")
    W, piv, _ = LU.getrf(Af, "fp16", 8)
    r = F.round_to(rng.standard_normal(n), "fp64")
    tr = []
    d, k = G.gmres(A, W, piv, None, r, "fp64", "fp64", tau=1e-10, k_max=n, trace=tr)
    assert 3 <= k < n
    assert tr[-1] <= 1e-10 and all(t > 1e-10 for t in tr[:-1])
    # true preconditioned residual of the result is consistent with the estimate
    Minv = lambda v: np.linalg.solve((np.tril(W, -1) + np.eye(n)) @ np.triu(W), v[LU.perm_from_piv(piv)])
    c = Minv(r)
    res = np.linalg.norm(c - Minv(A @ d)) / np.linalg.norm(c)
    assert res <= 1e-8
    # GMRES minimises the preconditioned residual over the Krylov space: compare
    # with an explicit least-squares solve over the same space.
    K = np.empty((n, k))
    v = c / np.linalg.norm(c)
    for j in range(k):
        K[:, j] = v
        v = Minv(A @ v)
        for i in range(j + 1):
            v -= (K[:, i] @ v) * K[:, i]
        v /= np.linalg.norm(v)
    y, *_ = np.linalg.lstsq(np.column_stack([Minv(A @ K[:, j]) for j in range(k)]), c, rcond=None)
    np.testing.assert_allclose(d, K @ y, rtol=0, atol=1e-8 * np.abs(d).max())


def test_gmres_restart_beyond_count_is_identical():
    n = 30
    rng = np.random.default_rng(4)
    A = rng.standard_normal((n, n)) + 3 * np.eye(n)
    W, piv, _ = LU.getrf(F.round_to(A, "fp16"), "fp16", 8)
    r = F.round_to(rng.standard_normal(n), "fp32")
    d1, k1 = G.gmres(A, W, piv, None, r, "fp32", "fp32", 1e-6, 20, restart=0)
    d2, k2 = G.gmres(A, W, piv, None, r, "fp32", "fp32", 1e-6, 20, restart=25)
    assert k1 == k2
    np.testing.assert_array_equal(d1, d2)
    d3, k3 = G.gmres(A, W, piv, None, r, "fp32", "fp32", 1e-6, 20, restart=2)
    assert k3 >= k1
    want = np.linalg.solve(A, r)
    assert np.abs(d3 - want).max() <= 1e-4 * np.abs(want).max()


def test_gmres_caps_iterations():
    n = 50
    rng = np.random.default_rng(5)
    A = rng.standard_normal((n, n))
    W, piv, _ = LU.getrf(F.round_to(A + rng.standard_normal((n, n)), "fp16"), "fp16", 8)
    r = F.round_to(rng.standard_normal(n), "fp32")
    d, k = G.gmres(A, W, piv, None, r, "fp32", "fp32", 1e-12, 7.3)
    assert k == 8     # ceil(k_max)

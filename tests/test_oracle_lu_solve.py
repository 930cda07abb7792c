"""Pins for the oracle's LU (Alg. 4 first line) and triangular solves.

What fixes the expected values here is independent of the oracle's code:
LAPACK (scipy) for float64 factors and pivots, Higham's componentwise backward
error bound |PA - LU| <= gamma |L||U| for Gaussian elimination, matrices whose
pivot sequence is known in closed form, exact rational arithmetic on tiny
inputs, and integer triangular systems whose solves are exact.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fmt as F
from oracle import lu as LU
from oracle import solve as SV
from oracle import scaling as SC


def rand(n, seed=0):
    return np.random.default_rng(seed).standard_normal((n, n))


@pytest.mark.parametrize("n,nb", [(9, 4), (33, 8), (64, 64), (70, 16)])
def test_fp64_matches_lapack(n, nb):
    A = rand(n, n)
    W, piv, info = LU.getrf(A, "fp64", nb)
    lu, lpiv = sla.lu_factor(A)
    assert info == 0
    np.testing.assert_array_equal(piv, lpiv)
    np.testing.assert_allclose(W, lu, rtol=0, atol=1e-12 * np.abs(lu).max())


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32"])
@pytest.mark.parametrize("n,nb", [(40, 8), (96, 16), (130, 32)])
def test_backward_error_bound(fmt, n, nb):
    # Higham, Thm 9.3: |PA - LU| <= gamma_n |L||U|; storage in u_f each update step
    # contributes at most one u_f rounding per step, so gamma uses (n/nb + 3) u_f.
    A = F.round_to(rand(n, 1) * 8, fmt)
    W, piv, info = LU.getrf(A, fmt, nb)
    L, U = LU.unpack(W)
    p = LU.perm_from_piv(piv)
    E = np.abs(A[p] - L @ U)
    g = (n / nb + n * F.u("fp32") / F.u(fmt) + 3) * F.u(fmt)
    bound = g / (1 - g) * (np.abs(L) @ np.abs(U))
    assert np.all(E <= bound + 1e-300)
    assert np.all(np.abs(np.tril(W, -1)) <= 1.0)      # partial pivoting: |l_ij| <= 1


def manufactured(n, order, seed=0):
    """Matrix whose GEPP pivot at step k is row order[k]: entry order[k] of column k
    dominates everything below by a margin that no rounding can overturn."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1, 1, (n, n)) * 2.0 ** -8
    for k, r in enumerate(order):
        A[r, k] = 2.0 ** (12 - k % 4) * (1 if k % 2 else -1)
    return A


@pytest.mark.parametrize("fmt", ["fp16", "fp32", "fp64"])
def test_manufactured_pivots(fmt):
    n = 48
    order = list(np.random.default_rng(5).permutation(n))
    A = F.round_to(manufactured(n, order), fmt)
    W, piv, info = LU.getrf(A, fmt, 16)
    # expected LAPACK interchanges for a pivot row known in original numbering
    pos = list(range(n))      # pos[i] = original row currently at position i
    want = []
    for k, r in enumerate(order):
        p = pos.index(r)
        want.append(p)
        pos[k], pos[p] = pos[p], pos[k]
    assert list(piv) == want


def test_ties_and_nan_and_zero_pivot():
    # first index wins on ties; NaN never wins; an all-zero column gives info
    A = np.array([[1.0, 2.0, 0.0], [-1.0, 1.0, 0.0], [0.5, np.nan, 0.0]])
    W, piv, info = LU.getrf(A, "fp32", 3)
    assert piv[0] == 0          # |1| == |-1|: first index
    assert info == 3            # third column zero below the diagonal
    B = np.array([[np.nan, 1.0], [2.0, 1.0]])
    W, piv, info = LU.getrf(B, "fp32", 2)
    assert piv[0] == 1


def test_tiny_lu_against_rationals():
    """nb=1 fp32 elimination on a 4x4: every operation re-executed with Fractions
    and rounded explicitly (reciprocal rounded, product rounded, fma rounded once)."""
    rng = np.random.default_rng(2)
    A = F.round_to(rng.standard_normal((4, 4)), "fp32")
    W, piv, info = LU.getrf(A, "fp32", 4)
    M = [[Fraction(v) for v in row] for row in A]
    n = 4

    def r32(fr):
        return Fraction(float(F.round_to(np.array([float(fr)]), "fp32")[0])) if abs(float(fr)) > 1e-30 else Fraction(0)

    def fma_r(a, b, c):
        from tests.test_oracle_fmt import exact_round_fraction
        return Fraction(exact_round_fraction(a * b + c))

    for k in range(n):
        p = max(range(k, n), key=lambda i: (abs(M[i][k]), -i))
        M[k], M[p] = M[p], M[k]
        assert piv[k] == p
        rcp = r32(1 / M[k][k])
        for i in range(k + 1, n):
            M[i][k] = r32(M[i][k] * rcp)
            for j in range(k + 1, n):
                M[i][j] = fma_r(-M[i][k], M[k][j], M[i][j])
    np.testing.assert_array_equal(W, np.array([[float(v) for v in row] for row in M]))


def test_solve_fp64_matches_lapack():
    n = 57
    A = rand(n, 3)
    W, piv, info = LU.getrf(A, "fp64", 8)
    b = np.random.default_rng(4).standard_normal(n)
    y = SV.lu_solve(W, piv, b, "fp64")
    want = sla.lu_solve(sla.lu_factor(A), b)
    np.testing.assert_allclose(y, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_solve_exact_on_integer_triangles():
    # unit lower L and upper U with integer entries, pivots powers of two, small
    # integer right-hand side: every intermediate is an exactly representable
    # integer/dyadic, so the fp16 substitution must return the exact solution.
    n = 6
    L = np.eye(n) + np.tril(np.ones((n, n)), -1)
    U = np.triu(np.ones((n, n))) + np.diag([1.0, 1.0, 3.0, 1.0, 1.0, 1.0]) * 0
    U[np.diag_indices(n)] = [2.0, 4.0, 1.0, 2.0, 8.0, 1.0]
    x = np.array([1.0, -2.0, 3.0, 0.5, -1.0, 2.0])
    b = L @ (U @ x)
    W = np.tril(L, -1) + U
    y = SV.lu_solve(W, np.arange(n), b, "fp16")
    np.testing.assert_array_equal(y, x)


def test_solve_fp16_components_overflow_to_inf():
    # a solution component above 65504 must become +inf in the u_f = fp16 solve
    W = np.array([[2.0 ** -10, 0.0], [0.0, 1.0]])
    y = SV.lu_solve(W, np.arange(2), np.array([100.0, 1.0]), "fp16")
    assert y[0] == math.inf and y[1] == 1.0


def test_solve_tiny_against_rationals():
    """u_f = fp16 substitution on a 5x5 re-executed in exact arithmetic, each
    component rounded to fp16 (float64 accumulation is exact here)."""
    rng = np.random.default_rng(9)
    n = 5
    W = F.round_to(rng.uniform(-1, 1, (n, n)), "fp16")
    W[np.diag_indices(n)] = F.round_to(rng.uniform(1, 2, n), "fp16")
    piv = np.array([2, 1, 4, 3, 4])
    t = rng.standard_normal(n)
    y = SV.lu_solve(W, piv, t, "fp16")
    v = [Fraction(float(a)) for a in t]
    for j, k in enumerate(piv):
        v[j], v[k] = v[k], v[j]
    r16 = lambda fr: Fraction(float(np.float16(float(fr))))
    v = [r16(a) for a in v]
    for i in range(n):
        v[i] = r16(v[i] - sum(Fraction(W[i, k]) * v[k] for k in range(i)))
    inv = [Fraction(1.0 / W[i, i]) for i in range(n)]
    for i in range(n - 1, -1, -1):
        v[i] = r16((v[i] - sum(Fraction(W[i, k]) * v[k] for k in range(i + 1, n))) * inv[i])
    np.testing.assert_array_equal(y, np.array([float(a) for a in v]))


def test_solve_dd_accuracy():
    # double-double solve with an exact fp64 LU of a well-conditioned matrix is
    # accurate far below float64 roundoff: check against a Fraction solve.
    n = 6
    A = rand(n, 6) + 4 * np.eye(n)
    W, piv, info = LU.getrf(A, "fp64", 6)
    t = np.random.default_rng(8).standard_normal(n)
    hi, lo = SV.lu_solve(W, piv, t, "dd")
    L, U = LU.unpack(W)
    p = LU.perm_from_piv(piv)
    # exact solution of (LU) y = P t with the stored factors
    M = [[Fraction(v) for v in row] for row in (L @ np.eye(n))]
    Lf = [[Fraction(L[i, j]) for j in range(n)] for i in range(n)]
    Uf = [[Fraction(U[i, j]) for j in range(n)] for i in range(n)]
    v = [Fraction(t[p[i]]) for i in range(n)]
    for i in range(n):
        v[i] -= sum(Lf[i][k] * v[k] for k in range(i))
    for i in range(n - 1, -1, -1):
        v[i] = (v[i] - sum(Uf[i][k] * v[k] for k in range(i + 1, n))) / Uf[i][i]
    for i in range(n):
        err = abs(Fraction(hi[i]) + Fraction(lo[i]) - v[i])
        assert err <= abs(v[i]) * Fraction(2) ** -95


def test_scaling_is_power_of_two_and_exact():
    A = rand(30, 12) * np.exp2(np.random.default_rng(1).integers(-20, 20, (30, 1)))
    R, S, mu = SC.compute(A, "fp16", rows=True)
    for v in list(R) + list(S) + [mu]:
        m, e = math.frexp(v)
        assert m == 0.5
    As = SC.apply(A, R, S, mu)
    # exact: undoing the scaling recovers A bit for bit
    np.testing.assert_array_equal((As / mu) / S[None, :] / R[:, None], A)
    assert np.abs(As).max() <= SC.THETA * 65504 and np.abs(As).max() > SC.THETA * 65504 / 2
    # rows (then columns) have maxima in [1/2, 1) before mu
    RA = np.abs(A) * R[:, None]
    assert np.all((RA.max(axis=1) >= 0.5) & (RA.max(axis=1) < 1))


@pytest.mark.parametrize("fmt,n,nb", [("fp16", 100, 16), ("fp32", 70, 8), ("fp64", 50, 4)])
def test_exact_factors_recovered(fmt, n, nb):
    # A = P0^T L0 U0 with dyadic multipliers |l| <= 1/2 and a power-of-two diagonal:
    # all arithmetic is exact, so GEPP must return exactly (P0, L0, U0).
    rng = np.random.default_rng(n)
    L0 = np.tril(rng.choice([0.0, 0.25, -0.25, 0.5, -0.5], (n, n)), -1) + np.eye(n)
    U0 = np.triu(rng.integers(-4, 5, (n, n)).astype(float), 1)
    U0[np.diag_indices(n)] = rng.choice([1.0, -1.0, 2.0, -2.0, 4.0, -4.0, 8.0, -8.0], n)
    P0 = rng.permutation(n)
    A = np.empty((n, n))
    A[P0] = L0 @ U0
    W, piv, info = LU.getrf(A, fmt, nb)
    np.testing.assert_array_equal(W, np.tril(L0, -1) + U0)
    p = LU.perm_from_piv(piv)
    np.testing.assert_array_equal(p, P0)

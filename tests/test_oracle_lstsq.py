"""Pins of the least-squares oracle (augmented-system MSIR; Sec. 4 future work).

Each test fixes the oracle against something it does not compute itself: the
least-squares solution built into the generator, numpy's SVD-based lstsq, the
normal equations solved exactly in rationals, and the structure of the augmented
matrix."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import lstsq as OL
from oracle import msir as OM
from paper_2107_06200_amd import workloads as WL


def test_alpha_default_is_the_largest_power_of_two_below_max_abs():
    for amax, want in [(3.0, 2.0), (0.75, 0.5), (1.0, 1.0), (4.0, 4.0), (1e-3, 2.0 ** -10)]:
        A = np.array([[amax, -0.1 * amax], [0.2 * amax, -0.3 * amax]])
        assert OL.alpha_default(A) == want
    assert OL.alpha_default(np.zeros((3, 2))) == 1.0


def test_augmented_matrix_structure():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((5, 3))
    b = rng.standard_normal(5)
    K, f = OL.augment(A, b, 0.5)
    assert K.shape == (8, 8) and np.array_equal(K, K.T)
    assert np.array_equal(K[:5, :5], 0.5 * np.eye(5))
    assert np.array_equal(K[:5, 5:], A) and np.array_equal(K[5:, :5], A.T)
    assert np.array_equal(K[5:, 5:], np.zeros((3, 3)))
    assert np.array_equal(f, np.concatenate([b, np.zeros(3)]))


@pytest.mark.parametrize("m,n,kappa,scale", [(30, 12, 10.0, 8.0), (40, 25, 100.0, 0.3)])
def test_solution_and_residual_of_a_generated_problem(m, n, kappa, scale):
    A, x_t, b, r_t = WL.ls_system(m, n, kappa, 3, np.random.default_rng(m), rnorm=1e-2)
    A, b, r_t = A * scale, b * scale, r_t * scale
    x, r, alpha, res = OL.lstsq(A, b)
    assert res.cged
    assert alpha == OL.alpha_default(A) and alpha != 1.0
    # the generator's solution and numpy's SVD-based solution (independent routes)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    tol = 1e-13 * kappa ** 2
    assert np.max(np.abs(x - x_t)) <= tol * np.max(np.abs(x_t))
    assert np.max(np.abs(x - xs)) <= tol * np.max(np.abs(xs))
    assert np.max(np.abs(r - r_t)) <= tol * np.max(np.abs(b))
    # optimality: A^T r = 0 and r = b - A x, both up to rounding
    assert np.max(np.abs(A.T @ r)) <= 1e-13 * np.abs(A).max() * np.abs(r).max() * m
    assert np.max(np.abs(r - (b - A @ x))) <= 1e-13 * np.abs(b).max()


def test_square_case_is_the_linear_solve():
    A, x_t, b = WL.randsvd(20, 10.0, 3, np.random.default_rng(3))
    x, r, _, res = OL.lstsq(A, b)
    assert res.cged
    assert np.max(np.abs(x - np.linalg.solve(A, b))) <= 1e-12 * np.abs(x_t).max()
    assert np.max(np.abs(r)) <= 1e-13 * np.abs(b).max()


def test_tiny_problem_against_exact_normal_equations():
    A = np.array([[1.0, 2.0], [3.0, -1.0], [2.0, 5.0]])
    b = np.array([4.0, -2.0, 7.0])
    # exact x from A^T A x = A^T b (Cramer's rule in rationals)
    Af = [[Fraction(int(v)) for v in row] for row in A]
    bf = [Fraction(int(v)) for v in b]
    G = [[sum(Af[k][i] * Af[k][j] for k in range(3)) for j in range(2)] for i in range(2)]
    c = [sum(Af[k][i] * bf[k] for k in range(3)) for i in range(2)]
    det = G[0][0] * G[1][1] - G[0][1] * G[1][0]
    xe = [(c[0] * G[1][1] - G[0][1] * c[1]) / det, (G[0][0] * c[1] - c[0] * G[1][0]) / det]
    x, r, alpha, res = OL.lstsq(A, b)
    assert alpha == 4.0
    for xi, ei in zip(x, xe):
        assert abs(xi - float(ei)) <= 1e-14 * abs(float(ei))
    re = [bf[k] - Af[k][0] * xe[0] - Af[k][1] * xe[1] for k in range(3)]
    for ri, ei in zip(r, re):
        assert abs(ri - float(ei)) <= 1e-14 * max(abs(float(e)) for e in re)


def test_ill_conditioned_problem_goes_through_the_stages():
    # kappa(A) = 1e4 with alpha = sigma_min / sqrt(2) (power of two): the augmented
    # system has condition about 2 kappa, beyond fp16 SIR, and Alg. 4 still reaches x
    m, n, kappa = 60, 20, 1e4
    A, x_t, b, r_t = WL.ls_system(m, n, kappa, 3, np.random.default_rng(7), rnorm=1e-3)
    a = 2.0 ** round(np.log2(1.0 / kappa / np.sqrt(2.0)))
    x, r, alpha, res = OL.lstsq(A, b, OM.Params(scaling="auto"), alpha=a)
    assert alpha == a and res.cged
    assert any(s.stage != 0 for s in res.history) or res.n_lu > 1
    assert np.max(np.abs(x - x_t)) <= 1e-13 * kappa ** 2 * np.abs(x_t).max()


def test_rejects_wide_matrices():
    with pytest.raises(ValueError):
        OL.lstsq(np.ones((2, 3)), np.ones(2))

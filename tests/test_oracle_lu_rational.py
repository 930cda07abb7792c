"""Bit-level pins of the oracle's blocked LU (DM(nb)), its scaling and the fp32 A v.

The blocked LU of Alg. 4's first line (factors stored in u_f, arithmetic in fp32) is
re-executed here from its definition with exact rational arithmetic, every rounding
being applied explicitly (round to nearest, ties to even, written from the
definition with fractions.Fraction) and in the order the definition fixes:

  per panel of nb columns: pivot = first row of largest magnitude; reciprocal of the
  pivot rounded to fp32; multipliers = fl32(l * rcp); rank-1 updates as single-rounded
  fp32 fused multiply-adds; the panel rounded to u_f when written back; U12 by forward
  substitution with single-rounded fp32 fused multiply-adds, row c using rows 0..c-1
  in increasing order, then rounded to u_f; the trailing block as a sequential chain
  of single-rounded fp32 fused multiply-adds over the panel's columns (k ascending),
  then rounded to u_f.

Sizes n = 6..8 with nb in {2, 4} (several panels, several trailing updates) in fp16,
bf16 and fp32, fp16 also with the power-of-two scaling of Sec. 2.1.2.  Each plausible
slip in the oracle (U12 left unrounded, multiply-adds rounded twice, the trailing chain
in another order or summed exactly before one rounding, the write-back to u_f skipped)
is re-executed too, and the test inputs are checked to tell every such variant apart
from the definition, so a slip of that kind in the oracle would fail the pin.  A
one-ulp fp32 difference in the chain survives the final rounding to fp16 or bf16 only
near a tie of that format, so the chain's rounding and order are told apart by the
fp32-factor cases, which run the same code of the oracle (arithmetic format fp32,
sequential chain); the u_f roundings by the fp16 and bf16 cases.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import fmt as F
from oracle import lu as LU
from oracle import ops as OPS
from oracle import scaling as SC

# (significand bits incl. the hidden one, minimum normal exponent, largest finite value)
_SPEC = {"fp16": (11, -14, Fraction(65504)),
         "bf16": (8, -126, Fraction(2) ** 127 * (2 - Fraction(1, 2 ** 7))),
         "fp32": (24, -126, Fraction(2) ** 127 * (2 - Fraction(1, 2 ** 23)))}


def rnd(X, fmt):
    """Nearest value of ``fmt`` to the rational X, ties to the even significand.
    (Magnitudes beyond the largest finite value would round to infinity; the inputs
    below stay far from that, which the assertion checks.)"""
    if X == 0:
        return Fraction(0)
    p, emin, xmax = _SPEC[fmt]
    a = abs(X)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q = Fraction(2) ** (max(e, emin) - (p - 1))
    lo = (a // q) * q
    hi = lo + q
    if a - lo < hi - a or (a - lo == hi - a and (lo / q) % 2 == 0):
        r = lo
    else:
        r = hi
    assert r <= xmax
    return r if X > 0 else -r


def lu_rational(A, fmt_f, nb, round_u12=True, fma_single=True, writeback=True, k_ascending=True,
                trail_chain=True):
    """DM(nb) on a float64 matrix whose entries are u_f values; returns (W, piv) as
    float64.  The keyword switches re-execute the slips listed in the module text."""
    n = A.shape[0]
    W = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(n)]
    piv = list(range(n))
    r32 = lambda x: rnd(x, "fp32")
    rf = (lambda x: rnd(x, fmt_f)) if writeback else (lambda x: x)

    def fma(a, b, c):        # fl32(a * b + c): one rounding, or two for the slip
        return r32(a * b + c) if fma_single else r32(r32(a * b) + c)

    for j0 in range(0, n, nb):
        jb = min(nb, n - j0)
        cols = range(j0, j0 + jb)
        for c in cols:
            p = max(range(c, n), key=lambda r: (abs(W[r][c]), -r))
            piv[c] = p
            W[c], W[p] = W[p], W[c]          # whole rows: inside and outside the panel
            if W[c][c] == 0:
                continue
            rcp = r32(1 / W[c][c])
            for r in range(c + 1, n):
                W[r][c] = r32(W[r][c] * rcp)
                for k in range(c + 1, j0 + jb):
                    W[r][k] = fma(-W[r][c], W[c][k], W[r][k])
        for r in range(j0, n):
            for k in cols:
                W[r][k] = rf(W[r][k])
        right = range(j0 + jb, n)
        for c in range(j0 + 1, j0 + jb):                     # U12 by forward substitution
            for k in range(j0, c):
                for j in right:
                    W[c][j] = fma(-W[c][k], W[k][j], W[c][j])
        if round_u12:
            for c in cols:
                for j in right:
                    W[c][j] = rf(W[c][j])
        for r in range(j0 + jb, n):                          # trailing update
            for j in right:
                if trail_chain:
                    acc = W[r][j]
                    for k in (cols if k_ascending else reversed(cols)):
                        acc = fma(-W[r][k], W[k][j], acc)
                else:                                        # slip: exact sum rounded once
                    acc = r32(W[r][j] - sum(W[r][k] * W[k][j] for k in cols))
                W[r][j] = rf(acc)
    return np.array([[float(v) for v in row] for row in W]), np.array(piv)


def case(n, fmt, scaled, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) * np.exp2(rng.integers(-3, 4, (n, 1)))
    if scaled:
        A = SC.apply(A, *SC.compute(A, fmt, rows=True))
    return F.round_to(A, fmt)


CASES = [(n, nb, fmt, scaled, seed)
         for (n, nb) in ((6, 2), (7, 2), (8, 4), (8, 2))
         for fmt in ("fp16", "bf16", "fp32")
         for scaled in (False, True)
         for seed in (1, 2)
         if not (scaled and fmt != "fp16")]


@pytest.mark.parametrize("n,nb,fmt,scaled,seed", CASES)
def test_blocked_lu_bit_exact_against_rationals(n, nb, fmt, scaled, seed):
    A = case(n, fmt, scaled, seed)
    W, piv, info = LU.getrf(A, fmt, nb)
    Wq, pq = lu_rational(A, fmt, nb)
    assert info == 0
    np.testing.assert_array_equal(piv, pq)
    np.testing.assert_array_equal(W, Wq)


@pytest.mark.parametrize("slip", ["round_u12", "fma_single", "writeback", "k_ascending", "trail_chain"])
def test_pin_detects_each_slip(slip):
    # each slip, re-executed, differs from the definition on at least one of the
    # pinned cases, so an oracle containing it could not pass the test above
    differs = 0
    for n, nb, fmt, scaled, seed in CASES:
        A = case(n, fmt, scaled, seed)
        Wq, pq = lu_rational(A, fmt, nb)
        Ws, ps = lu_rational(A, fmt, nb, **{slip: False})
        differs += int(not (np.array_equal(Wq, Ws) and np.array_equal(pq, ps)))
    assert differs >= 3, (slip, differs)


@pytest.mark.parametrize("rows", [True, False])
def test_column_scaling_maxima(rows):
    # Sec. 2.1.2 scaling: after R (rows) and S (columns) every column of |R A S| has its
    # largest entry in [1/2, 1), every row of |R A| too when rows are equilibrated,
    # and mu puts the largest entry of mu R A S in (theta xmax / 2, theta xmax]
    rng = np.random.default_rng(11)
    A = rng.standard_normal((25, 25)) * np.exp2(rng.integers(-30, 30, (25, 1))) \
        * np.exp2(rng.integers(-10, 10, (1, 25)))
    R, S, mu = SC.compute(A, "fp16", rows=rows)
    if not rows:
        assert np.all(R == 1.0)
    cm = (np.abs(A) * R[:, None] * S[None, :]).max(axis=0)
    assert np.all((cm >= 0.5) & (cm < 1.0))
    m = np.abs(SC.apply(A, R, S, mu)).max()
    assert SC.THETA * 65504 / 2 < m <= SC.THETA * 65504


def test_fp32_matvec_is_rounded_once_from_the_exact_product():
    # A v in fp32 (the SGMRES-IR operator's product): A and v rounded to fp32, the sum of
    # products formed in float64 and rounded to fp32.  Against the exact rational product
    # rounded once: equal except where the float64 sum falls within 2^-53 of an fp32
    # tie (probability ~2^-29 per entry), which these inputs do not hit.
    rng = np.random.default_rng(12)
    n = 9
    for t in range(40):
        A = rng.standard_normal((n, n)) * np.exp2(rng.integers(-6, 6, (n, n)))
        v = rng.standard_normal(n)
        got = OPS.matvec(A, v, "fp32")
        Au = [[Fraction(float(x)) for x in row] for row in F.round_to(A, "fp32")]
        vu = [Fraction(float(x)) for x in F.round_to(v, "fp32")]
        want = [float(rnd(sum(Au[i][j] * vu[j] for j in range(n)), "fp32")) for i in range(n)]
        np.testing.assert_array_equal(got, np.array(want))

"""Pins for the oracle's formats and rounding (Table 3; IEEE round-to-nearest-even).

Each rounding is checked against exact rational arithmetic (fractions.Fraction),
an independent definition of "the representable value nearest to x, ties to the
even significand"; numpy's own float16/float32 casts are a second, library
reference for those two formats.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import fmt as F

SPEC = {"fp16": (11, -14, 65504.0), "bf16": (8, -126, F.XMAX["bf16"]), "fp32": (24, -126, F.XMAX["fp32"])}


def exact_round(x, fmt):
    """Round a float64 to fmt with Fractions: enumerate the two neighbours."""
    p, emin, xmax = SPEC[fmt]
    if math.isnan(x) or math.isinf(x) or x == 0.0:
        return x
    X = Fraction(x)
    a = abs(X)
    e = math.floor(math.log2(a))
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, emin)
    q = Fraction(2) ** (e - (p - 1))
    lo = (a // q) * q
    hi = lo + q
    if a - lo < hi - a:
        r = lo
    elif a - lo > hi - a:
        r = hi
    else:
        r = lo if (lo / q) % 2 == 0 else hi
    # overflow: beyond xmax + half an ulp of xmax rounds to infinity
    if r > Fraction(xmax):
        return math.copysign(math.inf, x)
    return math.copysign(float(r), x)


def test_table3_unit_roundoffs():
    # Table 3 prints 4.88e-4, 5.96e-8, 1.11e-16, 9.63e-35
    for f, printed in (("fp16", 4.88e-4), ("fp32", 5.96e-8), ("fp64", 1.11e-16), ("quad", 9.63e-35)):
        assert float(f"{F.u(f):.2e}") == printed
    assert F.u("bf16") == 2.0 ** -8
    assert F.u("dd") == F.u("fp64") ** 2


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32"])
def test_round_matches_exact_rational(fmt):
    rng = np.random.default_rng(7)
    p, emin, xmax = SPEC[fmt]
    span = {"fp16": (-28, 17), "bf16": (-135, 128), "fp32": (-152, 128)}[fmt]
    x = rng.standard_normal(3000) * np.exp2(rng.uniform(*span, 3000))
    got = F.round_to(x, fmt)
    for xi, gi in zip(x, got):
        want = exact_round(float(xi), fmt)
        assert (gi == want) or (math.isnan(gi) and math.isnan(want)), (fmt, xi, gi, want)


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32"])
def test_round_edge_cases(fmt):
    p, emin, xmax = SPEC[fmt]
    ulp_max = 2.0 ** (math.floor(math.log2(xmax)) - (p - 1))
    sub = 2.0 ** (emin - (p - 1))
    cases = [0.0, -0.0, 1.0, xmax, xmax + ulp_max / 2, xmax + ulp_max / 2 * (1 - 2 ** -30),
             sub, sub / 2, sub / 2 * (1 + 2 ** -20), 1.5 * sub, 2.5 * sub,
             1.0 + 2.0 ** -p, 1.0 + 3 * 2.0 ** -p, 1.0 + 2.0 ** -p * (1 + 2 ** -30), -1.0 - 2.0 ** -p,
             math.inf, -math.inf]
    got = F.round_to(np.array(cases), fmt)
    for xi, gi in zip(cases, got):
        assert gi == exact_round(xi, fmt) or (math.isnan(gi) and math.isnan(exact_round(xi, fmt))), (xi, gi)
    assert math.isnan(F.round_to(np.array([np.nan]), fmt)[0])
    # tie to even at 1 + 2^-p (halfway between 1 and 1 + 2^(1-p)) goes down to 1
    assert F.round_to(np.array([1.0 + 2.0 ** -p]), fmt)[0] == 1.0
    # overflow threshold: xmax + ulp/2 is a tie whose even neighbour is 2^(emax+1) -> inf
    assert F.round_to(np.array([xmax + ulp_max / 2]), fmt)[0] == math.inf


@pytest.mark.parametrize("fmt,dt", [("fp16", np.float16), ("fp32", np.float32)])
def test_round_matches_numpy_casts(fmt, dt):
    rng = np.random.default_rng(11)
    x = rng.standard_normal(200000) * np.exp2(rng.uniform(-30, 17, 200000))
    with np.errstate(over="ignore"):
        want = x.astype(dt).astype(np.float64)
    np.testing.assert_array_equal(F.round_to(x, fmt), want)


def test_fma32_single_rounding_against_rationals():
    rng = np.random.default_rng(3)
    n = 3000
    a = F.round_to(rng.standard_normal(n), "fp32")
    b = F.round_to(rng.standard_normal(n), "fp32")
    c = F.round_to(rng.standard_normal(n) * np.exp2(rng.integers(-30, 30, n)), "fp32")
    # plant exact midpoint cases: c = -(a*b rounded to a 25-bit midpoint) + tiny
    got = F.fma32(a, b, c)
    for i in range(n):
        ex = float(Fraction(a[i]) * Fraction(b[i]) + Fraction(c[i]))
        # correct rounding of the exact value (computed from the rational, not via float64 sum)
        want = exact_round_fraction(Fraction(a[i]) * Fraction(b[i]) + Fraction(c[i]))
        assert got[i] == want, (a[i], b[i], c[i], got[i], want, ex)


def exact_round_fraction(X):
    if X == 0:
        return 0.0
    a = abs(X)
    e = math.floor(math.log2(float(a))) if float(a) > 0 else -200
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    q = Fraction(2) ** (e - 23)
    lo = (a // q) * q
    hi = lo + q
    if a - lo < hi - a:
        r = lo
    elif a - lo > hi - a:
        r = hi
    else:
        r = lo if (lo / q) % 2 == 0 else hi
    return float(r) if X > 0 else -float(r)


def test_fma32_midpoint_double_rounding_case():
    # a*b + c lands a hair above a binary32 midpoint; float64 rounding of the sum
    # would land exactly on the midpoint and round-half-even would go down.
    a = 1.0 + 2.0 ** -23            # binary32
    b = 1.0 + 2.0 ** -23
    # a*b = 1 + 2^-22 + 2^-46 exactly; take c = 2^-24 - 2^-22 so the sum is 1 + 2^-24 + 2^-46
    c = 2.0 ** -24 - 2.0 ** -22
    assert F.round_to(np.array([c]), "fp32")[0] == c
    exact = Fraction(a) * Fraction(b) + Fraction(c)
    assert F.fma32(a, b, c) == exact_round_fraction(exact) == 1.0 + 2.0 ** -23

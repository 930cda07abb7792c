"""Floating-point formats and round-to-nearest-even (oracle; test infrastructure only).

Unit roundoffs follow Table 3 of the paper (fp16 4.88e-4, fp32 5.96e-8,
fp64 1.11e-16, fp128 9.63e-35).  bfloat16 (mentioned as a future format in
Sec. 2.2 and Sec. 4) has 8 significand bits, u = 2^-8.  Quadruple precision is
stood in for by double-double ("dd"), whose unit roundoff 2^-106 equals the
square of fp64's, so the requirement u_r <= u^2 of Sec. 2 still holds.

``round_to(x, fmt)`` returns float64 values exactly representable in ``fmt``:
IEEE round-to-nearest, ties to even, gradual underflow, overflow to +-inf,
NaN preserved.  It is written from the definition (scale by a power of two so
that the target's quantum becomes 1, round to an integer with numpy's rint,
which is round-half-even, scale back), so every step is exact in float64.
"""
import numpy as np

# name -> (significand bits p incl. hidden bit, emin of normals, emax)
_SPEC = {
    "fp16": (11, -14, 15),
    "bf16": (8, -126, 127),
    "fp32": (24, -126, 127),
    "fp64": (53, -1022, 1023),
}

# Unit roundoff of each format (Table 3; bf16 and dd by definition).
UNIT_ROUNDOFF = {
    "fp16": 2.0 ** -11,
    "bf16": 2.0 ** -8,
    "fp32": 2.0 ** -24,
    "fp64": 2.0 ** -53,
    "dd": 2.0 ** -106,
    "quad": 2.0 ** -113,
}

# Largest finite value of each storable format.
XMAX = {
    "fp16": 65504.0,
    "bf16": float(np.ldexp(2.0 - 2.0 ** -7, 127)),
    "fp32": float(np.finfo(np.float32).max),
    "fp64": float(np.finfo(np.float64).max),
}

# Order used by the precision ladder (coarsest first).
LADDER = ["fp16", "bf16", "fp32", "fp64", "dd"]


def u(fmt):
    """Unit roundoff of ``fmt``."""
    return UNIT_ROUNDOFF[fmt]


def round_to(x, fmt):
    """Round float64 data to ``fmt`` (RNE), returned as float64.

    ``fmt`` == "fp64" or "dd" returns the input unchanged (it is already a
    float64 value; dd quantities are carried as explicit (hi, lo) pairs).
    """
    x = np.asarray(x, dtype=np.float64)
    if fmt in ("fp64", "dd"):
        return x.copy()
    p, emin, emax = _SPEC[fmt]
    out = np.array(x, dtype=np.float64, copy=True)
    finite = np.isfinite(out) & (out != 0.0)
    if not np.any(finite):
        return out
    v = out[finite]
    _, e = np.frexp(v)            # v = m * 2**e, 0.5 <= |m| < 1
    e = e - 1                     # v = m' * 2**e with 1 <= |m'| < 2
    e = np.maximum(e, emin)       # below the normal range the quantum is fixed
    q = e - (p - 1)               # exponent of the quantum (ulp) at v
    r = np.ldexp(np.rint(np.ldexp(v, -q)), q)
    big = np.abs(r) > XMAX[fmt]
    r[big] = np.copysign(np.inf, r[big])
    out[finite] = r
    return out


def is_representable(x, fmt):
    """True where ``x`` is exactly representable in ``fmt``."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        return (round_to(x, fmt) == x) | np.isnan(x)


def fma32(a, b, c):
    """Binary32 fused multiply-add, fl32(a*b + c) with a single rounding.

    a, b, c hold binary32 values (as float64).  a*b is exact in float64
    (24 + 24 <= 53 bits); the sum a*b + c is formed exactly as s + e by
    Knuth's TwoSum; the single rounding of s + e to binary32 equals the
    rounding of s unless s is exactly a binary32 midpoint and e != 0, in which
    case the tie is broken towards the sign of e.  (numpy's float64 -> float32
    cast is round-to-nearest-even; the tests pin it against rational rounding.)
    """
    a, b, c = np.broadcast_arrays(np.asarray(a, dtype=np.float64),
                                  np.asarray(b, dtype=np.float64),
                                  np.asarray(c, dtype=np.float64))
    shape = a.shape
    with np.errstate(all="ignore"):
        p = a * b
        s = p + c
        bb = s - p
        e = (p - (s - bb)) + (c - bb)
        r32 = s.astype(np.float32)
        r = r32.astype(np.float64)
        cand = (e != 0.0) & (r != s) & np.isfinite(s) & np.isfinite(r)
    if np.any(cand):
        rs, ss, es = r[cand], s[cand], e[cand]
        # the binary32 neighbour of rs on the far side of s
        away = np.nextafter(rs.astype(np.float32),
                            np.where(ss > rs, np.float32(np.inf), np.float32(-np.inf))).astype(np.float64)
        is_mid = (ss - rs) == (away - ss)
        lo = np.minimum(rs, away)
        hi = np.maximum(rs, away)
        r[cand] = np.where(is_mid, np.where(es > 0, hi, lo), rs)
    return r.reshape(shape)

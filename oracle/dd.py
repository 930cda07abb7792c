"""Double-double arithmetic (oracle; test infrastructure only).

Quadruple precision (u = 9.63e-35, Table 3) is used in the paper for u_r and for
the GMRES-IR operator when u = double.  Here it is stood in for by unevaluated
sums hi + lo of two float64 numbers (unit roundoff about 2^-106 = u_fp64^2).

The building blocks are error-free transformations: Knuth's TwoSum and
Dekker's TwoProduct with Veltkamp splitting (no fused multiply-add is used, so
numpy evaluates them exactly barring overflow).  Vectors are carried as pairs of
float64 arrays.
"""
import numpy as np

_SPLIT = 134217729.0  # 2**27 + 1


def two_sum(a, b):
    """s + e == a + b exactly, s = fl(a + b)."""
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def quick_two_sum(a, b):
    """Exact when |a| >= |b| (or a == 0)."""
    s = a + b
    e = b - (s - a)
    return s, e


def split(a):
    c = _SPLIT * a
    hi = c - (c - a)
    return hi, a - hi


def two_prod(a, b):
    """p + e == a * b exactly, p = fl(a * b) (Dekker)."""
    p = a * b
    ah, al = split(a)
    bh, bl = split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def add(ah, al, bh, bl):
    """(ah + al) + (bh + bl) in double-double (accurate, IEEE-style addition)."""
    s, e = two_sum(ah, bh)
    t, f = two_sum(al, bl)
    e = e + t
    s, e = quick_two_sum(s, e)
    e = e + f
    return quick_two_sum(s, e)


def add_d(ah, al, b):
    """(ah + al) + b with b a float64."""
    s, e = two_sum(ah, b)
    e = e + al
    return quick_two_sum(s, e)


def mul_d(ah, al, b):
    """(ah + al) * b with b a float64."""
    p, e = two_prod(ah, b)
    e = e + al * b
    return quick_two_sum(p, e)


def mul(ah, al, bh, bl):
    """(ah + al) * (bh + bl) in double-double."""
    p, e = two_prod(ah, bh)
    e = e + (ah * bl + al * bh)
    return quick_two_sum(p, e)


def div(ah, al, bh, bl):
    """(ah + al) / (bh + bl) in double-double (one Newton-style correction)."""
    q1 = ah / bh
    ph, pl = mul_d(bh, bl, q1)
    rh, rl = add(ah, al, -ph, -pl)
    q2 = rh / bh
    ph, pl = mul_d(bh, bl, q2)
    rh, rl = add(rh, rl, -ph, -pl)
    q3 = rh / bh
    s, e = quick_two_sum(q1, q2)
    return add_d(s, e, q3)


def to_float(ah, al):
    return ah + al

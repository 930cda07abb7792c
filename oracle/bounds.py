"""Condition-number limits for convergence (oracle; test infrastructure only).

Sec. 2.2: with u_f >= u and u_r <= u^2, both forward and normwise backward
errors converge to the level u when kappa_inf(A) is below
  SIR:        1 / u_f
  SGMRES-IR:  u^(-1/3) u_f^(-2/3)
  GMRES-IR:   u^(-1/2) u_f^(-1)
Table 4 lists these limits for five precision combinations using the unit
roundoffs of Table 3.
"""
from .fmt import UNIT_ROUNDOFF

# Table 3 values as printed (3 significant digits)
TABLE3 = {"fp16": 4.88e-4, "fp32": 5.96e-8, "fp64": 1.11e-16, "quad": 9.63e-35}


def limits(uf, u, table=TABLE3):
    """(SIR, SGMRES-IR, GMRES-IR) kappa_inf limits for unit roundoffs of formats uf, u."""
    a, b = table[uf], table[u]
    return (1.0 / a, b ** (-1.0 / 3.0) * a ** (-2.0 / 3.0), b ** -0.5 / a)


def limits_exact(uf, u):
    return limits(uf, u, UNIT_ROUNDOFF)

"""Multistage mixed precision iterative refinement, Alg. 4 (oracle; test infrastructure only).

The controller follows Alg. 4 of the paper with the stopping criteria of
Sec. 2.1.1 and the scalings of Sec. 2.1.2:

  factor A in u_f; x0 by substitution in u_f (x0 := 0 if it is not finite);
  loop: residual in u_r, scaled by its inf-norm and stored in u; a correction
  by SIR (triangular solves in u_f), SGMRES-IR (operator in u) or GMRES-IR
  (operator in u^2); x += ||r|| d; monitors z = ||d||/||x||,
  v = ||d_{i+1}||/||d_i||, rho_max, phi = z/(1 - rho_max); when a criterion
  fires and convergence is not detected, reset x to x0 if phi > phi_0, and move
  to the next variant; after GMRES-IR raise u_f to the next format with unit
  roundoff at most u_f^2, lower u to u_f if needed, u_r to u^2 if needed,
  refactor, and start again with SIR.

Readings used where the paper is silent or inconsistent (each listed with its
reason in the design notes of the repository):
  * x is stored in its own precision u_x (default fp64).  u_x = u reproduces
    Alg. 4 literally: x is stored in u, also after an escalation lowers u, so u_x
    then follows u.  The thresholds z <= u and phi <= sqrt(n) u use u_x.
  * monitors use the true correction delta = ||r||_inf ||d||_inf.
  * the iteration criterion is iter >= i_max; the GMRES criterion k >= k_max
    with GMRES capped at ceil(k_max) iterations.
  * a non-finite SIR correction switches to SGMRES-IR without updating x and
    without counting the step; a non-finite GMRES correction leaves x
    unchanged and moves to the next variant as an unconverged trigger.
  * at every switch iter, ||d_prev|| (= inf) and rho_max (= 0) are reset.
  * rho_max >= 1 gives phi = +inf (divergence).
  * x0 is computed once; phi_0 is the first phi computed.
  * the precision ladder is fp16/bf16 -> fp32 -> fp64; escalating beyond
    fp64 returns "not converged".
  * convergence detection: 'estimate' (0 <= phi <= sqrt(n) u_x, Alg. 4),
    'backward' (normwise backward error of the current x <= tol, checked at
    every residual; the metric of the throughput benchmark), 'true'
    (forward and normwise backward errors <= the initial u, the protocol of the
    paper's experiments), 'componentwise' (componentwise relative backward
    error <= tol, checked where 'backward' checks; Sec. 2.1.1 names
    componentwise measures as an alternative test).
"""
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import fmt as F
from . import lu as LU
from . import ops
from . import scaling as SC
from .gmres import gmres
from .solve import lu_solve

SIR, SGMRES, GMRES = 0, 1, 2
STAGE_NAMES = {SIR: "SIR", SGMRES: "SGMRES-IR", GMRES: "GMRES-IR"}

EV_NAN_D = 1        # non-finite correction
EV_RESET_X0 = 2     # x reset to x0
EV_SWITCH = 4       # next variant
EV_ESCALATE = 8     # factorization precision raised
EV_SCALED = 16      # the factorization in use was scaled
EV_NAN_X0 = 32      # x0 replaced by zero
EV_CONVERGED = 64


@dataclass
class Params:
    uf: str = "fp16"
    u: str = "fp32"
    ur: str = "fp64"
    ux: str = "fp64"
    i_max: int = 10
    tau: Optional[float] = None          # None: 1e-6 for u=fp32, 1e-10 for u=fp64
    rho_thresh: float = 0.5
    k_max: Optional[float] = None        # None: 0.1 n
    restart: int = 0
    conv: str = "backward"               # 'estimate' | 'backward' | 'true' | 'componentwise'
    tol_nbe: float = 1e-15
    scaling: str = "auto"                # 'never' | 'auto' | 'always' | 'cols'
    nb: Optional[int] = None            # None: the default width rule of oracle.lu.nb_auto
    max_steps: int = 1000
    lu_trailing: str = "fma32"          # 'fma32' | 'exact' (see oracle.lu.getrf)


@dataclass
class Step:
    level: int
    uf: str
    u: str
    ur: str
    stage: int
    iter: int
    k: int
    z: float
    v: float
    rho_max: float
    phi: float
    rnorm: float
    nbe: float
    events: int
    counted: bool = True


@dataclass
class Result:
    x: np.ndarray
    cged: bool
    status: int
    history: List[Step] = field(default_factory=list)
    n_lu: int = 0
    nbe: float = float("nan")
    ferr: float = float("nan")
    final: tuple = ()


class _LoggedList(list):
    """The history list; hands each appended step to ``log`` when one is given."""

    def __init__(self, log):
        super().__init__()
        self._log = log

    def append(self, step):
        super().append(step)
        if self._log is not None:
            self._log(step)


def next_uf(uf):
    """Next factorization format with unit roundoff <= u_f^2 (fp16/bf16 -> fp32 -> fp64)."""
    target = F.u(uf) ** 2
    for f in ("fp16", "bf16", "fp32", "fp64"):
        if F.u(f) <= target:
            return f
    return None


def square(uu):
    """The format whose unit roundoff is u^2 (fp32 -> fp64, fp64 -> dd)."""
    return {"fp32": "fp64", "fp64": "dd"}[uu]


def factor(A, uf, scaling_mode, nb, trailing="fma32"):
    """Alg. 4 first line with the Sec. 2.1.2 retry.  Returns (W, piv, info, scal, scaled)."""
    scal = None
    use_scaling = uf == "fp16" and scaling_mode in ("always", "cols")
    if use_scaling:
        scal = SC.compute(A, uf, rows=(scaling_mode == "always"))
        Af = F.round_to(SC.apply(A, *scal), uf)
    else:
        Af = F.round_to(A, uf)
    W, piv, info = LU.getrf(Af, uf, nb, trailing)
    if uf == "fp16" and scaling_mode == "auto" and not np.all(np.isfinite(W)):
        scal = SC.compute(A, uf, rows=True)
        Af = F.round_to(SC.apply(A, *scal), uf)
        W, piv, info = LU.getrf(Af, uf, nb, trailing)
    return W, piv, info, scal


def render(history):
    """The paper's notation, e.g. '2, (5,10), (10); 2, (2,2,2)' (Sec. 2, Table 2 text)."""
    levels = []
    cur = None
    for st in history:
        if cur is None or st.level != cur[0]:
            cur = (st.level, {SIR: 0, SGMRES: [], GMRES: []}, set())
            levels.append(cur)
        cur[2].add(st.stage)
        if st.stage == SIR:
            if st.counted:
                cur[1][SIR] += 1
        elif st.counted:
            cur[1][st.stage].append(st.k)
    parts = []
    for _, d, seen in levels:
        items = [str(d[SIR])]
        for s in (SGMRES, GMRES):
            if d[s]:
                items.append("(" + ",".join(str(k) for k in d[s]) + ")")
        parts.append(", ".join(items))
    return "; ".join(parts)


def msir(A, b, params=Params(), x_true=None, return_x0=False, correction=None, log=None):
    """Run Alg. 4 on A x = b.

    ``correction``: optional callable (stage, rhat, uf, u) -> (d, k) replacing the
    SIR / GMRES correction solvers (used to drive the controller with scripted
    sequences in tests); d is returned already in precision u.
    ``log``: optional callable receiving each history Step once it is complete
    (progress of long runs; it does not affect the computation).
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = A.shape[0]
    P = params
    uf, u, ur, ux = P.uf, P.u, P.ur, P.ux
    u0 = u
    ux_follows_u = P.ux == P.u          # Alg. 4 stores x in u
    k_max = 0.1 * n if P.k_max is None else P.k_max
    normA = float(np.abs(A).sum(axis=1).max())
    normb = float(np.abs(b).max())
    sqn = math.sqrt(n)
    hist = _LoggedList(log)
    level = 0
    n_lu = 1

    W, piv, info, scal = factor(A, uf, P.scaling, P.nb, P.lu_trailing)
    ev_scaled = EV_SCALED if scal is not None else 0
    x0 = lu_solve(W, piv, b, uf, scal)
    ev_pending = ev_scaled
    if not np.all(np.isfinite(x0)):
        x0 = np.zeros(n)
        ev_pending |= EV_NAN_X0
    x0 = F.round_to(x0, ux)
    x = x0.copy()
    phi0 = None
    alg = SIR
    it = 0
    dprev = math.inf
    rho_max = 0.0

    def tau_of(uu):
        if P.tau is not None:
            return P.tau
        return 1e-6 if uu == "fp32" else 1e-10

    def nbe_of(s, xx):
        den = normA * float(np.abs(xx).max()) + normb
        return s / den if den > 0 else (0.0 if s == 0 else math.inf)

    def errors_ok(xx, r):
        # The convergence test of the 'backward' and 'true' modes measures the
        # iterate's normwise backward error with an exactly rounded residual
        # (double-double), like the paper's experiments, which stop on the
        # computed errors rather than on the monitors.
        if P.conv not in ("backward", "true", "componentwise"):
            return False
        rt = r if isinstance(r, tuple) else ops.residual(A, xx, b, "dd")
        st = ops.rnorm_inf(rt)
        if not np.isfinite(st):
            return False
        if P.conv == "backward":
            return nbe_of(st, xx) <= P.tol_nbe
        if P.conv == "componentwise":
            # componentwise relative backward error (Sec. 2.1.2), tested where the
            # normwise one is: |r_i| from the double-double residual rounded once,
            # denominators (|A| |x| + |b|)_i in float64
            num = np.abs(rt[0] + rt[1])
            den = np.abs(A) @ np.abs(xx) + np.abs(b)
            with np.errstate(all="ignore"):
                q = np.where(den > 0, num / den, np.where(num > 0, np.inf, 0.0))
            return bool(q.max() <= P.tol_nbe)
        fe = float(np.abs(xx - x_true).max() / np.abs(x_true).max())
        return fe <= F.u(u0) and nbe_of(st, xx) <= F.u(u0)

    cached = None   # (x, r) of the last residual, reused while x is unchanged
    status = 1
    cged = False
    steps = 0
    while steps < P.max_steps:
        if cached is not None and cached[0] is x:
            r = cached[1]
        else:
            r = ops.residual(A, x, b, ur)
            cached = (x, r)
        s = ops.rnorm_inf(r)
        nbe_x = nbe_of(s, x) if np.isfinite(s) else math.nan
        if s == 0.0 or (P.conv in ("backward", "true", "componentwise") and np.isfinite(s) and errors_ok(x, r)):
            cged, status = True, 0
            break
        rhat = ops.scale_residual(r, s, u)
        it += 1
        steps += 1
        events = ev_pending
        ev_pending = 0
        k = -1
        if correction is not None:
            d, k = correction(alg, rhat, uf, u)
            d = np.asarray(d, dtype=np.float64)
        elif alg == SIR:
            d = F.round_to(lu_solve(W, piv, rhat, uf, scal), u)
        else:
            p = u if alg == SGMRES else square(u)
            d, k = gmres(A, W, piv, scal, rhat, u, p, tau_of(u), k_max, P.restart)
        if alg == SIR:
            if not np.all(np.isfinite(d)):
                # Alg. 4 NaN check: switch without updating x; the step is not counted.
                hist.append(Step(level, uf, u, ur, SIR, it, -1, math.nan, math.nan, rho_max, math.nan,
                                 s, nbe_x, events | EV_NAN_D | EV_SWITCH, counted=False))
                alg, it, dprev, rho_max = SGMRES, 0, math.inf, 0.0
                continue
        if not np.all(np.isfinite(d)):
            events |= EV_NAN_D
            trigger, conv_now = True, False
            z = v = phi = math.nan
        else:
            with np.errstate(all="ignore"):
                x_new = F.round_to(x + F.round_to(s * d, ux), ux)
                delta = s * float(np.abs(d).max())
                xn = float(np.abs(x).max())
                z = delta / xn if xn > 0 else (0.0 if delta == 0 else math.inf)
                v = delta / dprev if dprev != math.inf else 0.0
                rho_max = max(rho_max, v)
                phi = z / (1.0 - rho_max) if rho_max < 1.0 else math.inf
            if phi0 is None:
                phi0 = phi
            dprev = delta
            trigger = bool(z <= F.u(ux) or v >= P.rho_thresh or it >= P.i_max
                           or (alg != SIR and k >= k_max) or phi <= sqn * F.u(ux))
            x = x_new
            conv_now = False
            if trigger:
                if P.conv == "estimate":
                    conv_now = 0.0 <= phi <= sqn * F.u(ux)
                else:
                    r_new = ops.residual(A, x, b, ur)
                    cached = (x, r_new)
                    conv_now = errors_ok(x, r_new)
        rec = Step(level, uf, u, ur, alg, it, k, z, v, rho_max, phi, s, nbe_x, events)
        hist.append(rec)
        if trigger and conv_now:
            rec.events |= EV_CONVERGED
            cged, status = True, 0
            break
        if trigger:
            if phi0 is not None and phi > phi0:
                x = x0.copy()
                rec.events |= EV_RESET_X0
            it, dprev, rho_max = 0, math.inf, 0.0
            if alg == SIR:
                alg = SGMRES
                rec.events |= EV_SWITCH
            elif alg == SGMRES:
                alg = GMRES
                rec.events |= EV_SWITCH
            else:
                rec.events |= EV_ESCALATE
                nuf = next_uf(uf)
                if nuf is None:
                    status = 1
                    break
                uf = nuf
                if F.u(uf) < F.u(u):
                    u = uf
                if ux_follows_u:
                    ux = u                  # x keeps its values; later roundings use the new u
                if F.u(ur) > F.u(u) ** 2:
                    ur = square(u)
                level += 1
                W, piv, info, scal = factor(A, uf, P.scaling, P.nb, P.lu_trailing)
                n_lu += 1
                ev_pending = EV_SCALED if scal is not None else 0
                alg = SIR
    res = Result(x=x, cged=cged, status=status, history=list(hist), n_lu=n_lu)
    rr = ops.residual(A, x, b, "dd")
    res.nbe = float(ops.rnorm_inf(rr) / (normA * float(np.abs(x).max()) + normb)) if np.any(x) else math.nan
    if x_true is not None:
        res.ferr = float(np.abs(x - x_true).max() / np.abs(x_true).max())
    res.final = (uf, u, ur)
    if return_x0:
        return res, x0
    return res



def gmres_ir5(A, b, params=Params(), ug=None, up=None, x_true=None):
    """Five-precision GMRES-based refinement (GMRES-IR5 as summarised in Sec. 1).

    One LU factorization in u_f (the scaling policy of ``params``), x0 from the
    factors, then refinement steps: residual in u_r, the scaled residual rounded to
    the GMRES working precision u_g, GMRES in u_g with the preconditioned matrix
    applied in u_p, and the update x <- fl_ux(x + fl_ux(s d)).  There is no switching
    and no escalation: the solve stops when the convergence test of ``params.conv``
    passes ('estimate': 0 <= phi <= sqrt(n) u_x after each step; the other modes at
    every residual), on a non-finite correction, or after i_max steps.  With
    u_g = u_p = u this is SGMRES-IR (Alg. 3); u_g = u, u_p = u^2 is GMRES-IR (Alg. 2).
    Steps are recorded as GMRES-IR stage steps of level 0.
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = A.shape[0]
    P = params
    uf, u, ur, ux = P.uf, P.u, P.ur, P.ux
    ug = u if ug is None else ug
    up = square(u) if up is None else up
    k_max = 0.1 * n if P.k_max is None else P.k_max
    tau = P.tau if P.tau is not None else (1e-6 if ug == "fp32" else 1e-10)
    normA = float(np.abs(A).sum(axis=1).max())
    normb = float(np.abs(b).max())
    sqn = math.sqrt(n)

    def nbe_of(s, xx):
        den = normA * float(np.abs(xx).max()) + normb
        return s / den if den > 0 else (0.0 if s == 0 else math.inf)

    def errors_ok(xx):
        rt = ops.residual(A, xx, b, "dd")
        st = ops.rnorm_inf(rt)
        if not np.isfinite(st):
            return False
        if P.conv == "backward":
            return nbe_of(st, xx) <= P.tol_nbe
        if P.conv == "componentwise":
            num = np.abs(rt[0] + rt[1])
            den = np.abs(A) @ np.abs(xx) + np.abs(b)
            with np.errstate(all="ignore"):
                q = np.where(den > 0, num / den, np.where(num > 0, np.inf, 0.0))
            return bool(q.max() <= P.tol_nbe)
        if P.conv == "true":
            fe = float(np.abs(xx - x_true).max() / np.abs(x_true).max())
            return fe <= F.u(u) and nbe_of(st, xx) <= F.u(u)
        return False

    W, piv, info, scal = factor(A, uf, P.scaling, P.nb, P.lu_trailing)
    ev = EV_SCALED if scal is not None else 0
    x = lu_solve(W, piv, b, uf, scal)
    if not np.all(np.isfinite(x)):
        x = np.zeros(n)
        ev |= EV_NAN_X0
    x = F.round_to(x, ux)
    hist = []
    cged, status = False, 1
    dprev, rho_max = math.inf, 0.0
    for it in range(1, P.i_max + 1):
        r = ops.residual(A, x, b, ur)
        s = ops.rnorm_inf(r)
        nbe_x = nbe_of(s, x) if np.isfinite(s) else math.nan
        if s == 0.0 or (P.conv != "estimate" and np.isfinite(s) and errors_ok(x)):
            cged, status = True, 0
            break
        rhat = ops.scale_residual(r, s, ug)
        d, k = gmres(A, W, piv, scal, rhat, ug, up, tau, k_max, P.restart)
        d = np.asarray(d, dtype=np.float64)
        if not np.all(np.isfinite(d)):
            hist.append(Step(0, uf, u, ur, GMRES, it, k, math.nan, math.nan, rho_max, math.nan, s, nbe_x,
                             ev | EV_NAN_D))
            break
        with np.errstate(all="ignore"):
            x_new = F.round_to(x + F.round_to(s * d, ux), ux)
            delta = s * float(np.abs(d).max())
            xn = float(np.abs(x).max())
            z = delta / xn if xn > 0 else (0.0 if delta == 0 else math.inf)
            v = delta / dprev if dprev != math.inf else 0.0
            rho_max = max(rho_max, v)
            phi = z / (1.0 - rho_max) if rho_max < 1.0 else math.inf
        dprev = delta
        x = x_new
        rec = Step(0, uf, u, ur, GMRES, it, k, z, v, rho_max, phi, s, nbe_x, ev)
        ev = 0
        hist.append(rec)
        if P.conv == "estimate" and 0.0 <= phi <= sqn * F.u(ux):
            rec.events |= EV_CONVERGED
            cged, status = True, 0
            break
    else:
        # i_max steps done: the last iterate may still pass the test
        if P.conv != "estimate" and errors_ok(x):
            cged, status = True, 0
    res = Result(x=x, cged=cged, status=status, history=hist, n_lu=1)
    rr = ops.residual(A, x, b, "dd")
    res.nbe = float(ops.rnorm_inf(rr) / (normA * float(np.abs(x).max()) + normb)) if np.any(x) else math.nan
    if x_true is not None:
        res.ferr = float(np.abs(x - x_true).max() / np.abs(x_true).max())
    res.final = (uf, u, ur)
    return res

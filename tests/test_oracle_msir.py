"""Pins for the oracle's multistage controller (Alg. 4, Sec. 2.1.1, Table 4).

* Table 4: the closed forms of Sec. 2.2 with Table 3's unit roundoffs must
  reproduce all fifteen printed limits.
* The controller is driven with scripted corrections (a fake solver returning
  chosen correction sizes, NaNs and GMRES counts) and the transitions are
  derived by hand from Alg. 4 and the four criteria of Sec. 2.1.1.
* Convergence theory: kappa_inf * u_f << 1 keeps MSIR in SIR (Sec. 2.2); a
  problem far beyond 1/u_f makes SIR fail and MSIR move on.
* End to end: small systems against exact rational solutions.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import bounds, fmt as F, metrics, msir as M
from paper_2107_06200_amd import workloads as WL

TABLE4 = [  # (uf, u): SIR, SGMRES-IR, GMRES-IR as printed
    (("fp16", "fp32"), (2e3, 4e4, 8e6)),
    (("fp32", "fp32"), (2e7, 2e7, 7e10)),
    (("fp16", "fp64"), (2e3, 3e7, 2e11)),
    (("fp32", "fp64"), (2e7, 1e10, 2e15)),
    (("fp64", "fp64"), (9e15, 9e15, 9e23)),
]


@pytest.mark.parametrize("pair,printed", TABLE4)
def test_table4(pair, printed):
    got = bounds.limits(*pair)
    for g, p in zip(got, printed):
        assert float(f"{g:.0e}") == p, (pair, g, p)


def test_text_bounds_single_double_quad():
    # Sec. 1: (single, double, quad): SIR 2e7, SGMRES-IR 1e10, GMRES-IR 2e15
    s, sg, g = bounds.limits("fp32", "fp64")
    assert (float(f"{s:.0e}"), float(f"{sg:.0e}"), float(f"{g:.0e}")) == (2e7, 1e10, 2e15)


def small_system(n=20, seed=0, kappa=10.0):
    A, x, b = WL.randsvd(n, kappa, 3, WL.rng_for(99, seed))
    return A, x, b


class Script:
    """Fake correction solver: returns d = scale_i * rhat-shaped vectors."""

    def __init__(self, items):
        self.items = list(items)
        self.calls = []

    def __call__(self, stage, rhat, uf, u):
        kind, val, k = self.items.pop(0)
        self.calls.append(stage)
        n = len(rhat)
        if kind == "nan":
            return np.full(n, np.nan), k
        # correction with inf-norm val (relative to ||r||, because x += ||r|| d)
        d = np.zeros(n)
        d[0] = val
        return d, k


def run_script(items, **kw):
    A, x, b = small_system()
    p = M.Params(uf="fp16", u="fp32", ur="fp64", ux="fp64", conv="estimate", i_max=kw.pop("i_max", 10),
                 k_max=kw.pop("k_max", 5), **kw)
    s = Script(items)
    res = M.msir(A, b, p, correction=s)
    return res, s


def test_script_nan_first_sir_step_switches_without_counting():
    # Alg. 4 NaN check: "0, (...)": no SIR step counted; the next step is SGMRES-IR
    res, s = run_script([("nan", 0, -1), ("d", 1e-3, 5), ("d", 1e-9, 5)] + [("d", 1e-30, 5)] * 40, max_steps=6)
    assert s.calls[:2] == [M.SIR, M.SGMRES]
    assert res.history[0].counted is False and res.history[0].events & M.EV_NAN_D
    assert M.render(res.history).startswith("0, (5")


def test_script_kmax_switches_after_one_step():
    # fourth criterion: k >= k_max is detectable at once
    res, s = run_script([("nan", 0, -1), ("d", 1e-3, 5), ("d", 1e-6, 5), ("d", 1e-9, 5)] + [("d", 1e-30, 1)] * 40,
                        k_max=5, max_steps=5)
    assert s.calls[:4] == [M.SIR, M.SGMRES, M.GMRES, M.SIR]
    assert res.history[1].events & M.EV_SWITCH and res.history[2].events & M.EV_ESCALATE


def test_script_ratio_switch_after_two_steps():
    # v = ||d2||/||d1|| = 0.6 >= rho_thresh = 0.5 -> switch after the second step
    res, s = run_script([("d", 1e-3, -1), ("d", 0.6e-3, -1), ("d", 1e-6, 1)] + [("d", 1e-30, 1)] * 40,
                        max_steps=3)
    assert s.calls[:3] == [M.SIR, M.SIR, M.SGMRES]
    h = res.history
    assert h[1].events & M.EV_SWITCH
    assert abs(h[1].v - h[1].z * 0 - 0.6) < 0.05 or h[1].v >= 0.5


def test_script_imax():
    # third criterion iter >= i_max with steady contraction 0.1 (no other trigger)
    items = [("d", 1e-2 * 0.1 ** i, -1) for i in range(3)] + [("d", 1e-30, 1)] * 40
    res, s = run_script(items, i_max=3, max_steps=4)
    assert s.calls[:4] == [M.SIR, M.SIR, M.SIR, M.SGMRES]
    assert res.history[2].iter == 3 and res.history[2].events & M.EV_SWITCH


def test_script_reset_to_x0_on_divergence():
    # growing corrections: rho_max >= 1 gives phi = inf > phi_0: x is reset to x0
    res, s = run_script([("d", 1e-3, -1), ("d", 5e-3, -1), ("d", 1e-9, 1)] + [("d", 1e-30, 1)] * 40, max_steps=3)
    assert res.history[1].phi == math.inf
    assert res.history[1].events & M.EV_RESET_X0


def test_script_ladder_exhausted_not_converged():
    # every correction NaN in GMRES stages: the ladder fp16 -> fp32 -> fp64 is exhausted
    items = ([("nan", 0, -1)] + [("nan", 0, 5)] * 2) * 3
    res, s = run_script(items, max_steps=50)
    assert not res.cged and res.status == 1
    assert res.n_lu == 3


def test_render_notation():
    S = M.Step
    mk = lambda lvl, st, k, counted=True: S(lvl, "fp16", "fp32", "fp64", st, 1, k, 0, 0, 0, 0, 0, 0, 0, counted)
    h = [mk(0, M.SIR, -1), mk(0, M.SIR, -1), mk(0, M.SGMRES, 5), mk(0, M.SGMRES, 10), mk(0, M.GMRES, 10),
         mk(1, M.SIR, -1), mk(1, M.SIR, -1), mk(1, M.SGMRES, 2), mk(1, M.SGMRES, 2), mk(1, M.SGMRES, 2)]
    assert M.render(h) == "2, (5,10), (10); 2, (2,2,2)"
    h2 = [mk(0, M.SIR, -1, counted=False), mk(0, M.SGMRES, 10), mk(0, M.GMRES, 10), mk(1, M.SIR, -1)]
    assert M.render(h2) == "0, (10), (10); 1"


def test_well_conditioned_stays_in_sir():
    # kappa_inf u_f << 1 (Sec. 2.2, SIR limit 1/u_f): SIR alone converges to nbe <= 1e-15
    A, x, b = WL.randsvd(60, 5.0, 3, WL.rng_for(98, 0))
    assert WL.kappa_inf(A) * F.u("fp16") < 0.05
    res = M.msir(A, b, M.Params(uf="fp16", u="fp32", nb=16), x_true=x)
    assert res.cged and all(st.stage == M.SIR for st in res.history)
    assert res.nbe <= 1e-15


def test_ill_conditioned_leaves_sir():
    # kappa far above 1/u_f: SIR cannot converge; MSIR moves to a GMRES variant
    A, x, b = WL.randsvd(80, 1e7, 3, WL.rng_for(97, 0))
    res = M.msir(A, b, M.Params(uf="fp16", u="fp32", scaling="auto", nb=16), x_true=x)
    assert any(st.stage != M.SIR for st in res.history)
    assert res.cged and res.nbe <= 1e-15


def test_exact_rational_solution_small():
    # n = 6: x* = A^{-1} b exactly (Fractions); MSIR in backward mode reaches
    # ferr <= c kappa u_x and nbe <= 1e-15
    rng = np.random.default_rng(12)
    n = 6
    A = rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    res = M.msir(A, b, M.Params(uf="fp16", u="fp32", nb=4))
    Af = [[Fraction(v) for v in row] for row in A]
    bf = [Fraction(v) for v in b]
    # Gauss-Jordan in rationals
    Mx = [row[:] + [bf[i]] for i, row in enumerate(Af)]
    for k in range(n):
        p = max(range(k, n), key=lambda i: abs(Mx[i][k]))
        Mx[k], Mx[p] = Mx[p], Mx[k]
        for i in range(n):
            if i != k:
                f = Mx[i][k] / Mx[k][k]
                Mx[i] = [a - f * c for a, c in zip(Mx[i], Mx[k])]
    xs = np.array([float(Mx[i][n] / Mx[i][i]) for i in range(n)])
    kap = WL.kappa_inf(A)
    assert res.cged
    assert np.abs(res.x - xs).max() / np.abs(xs).max() <= 10 * kap * F.u("fp64")
    assert metrics.nbe(A, res.x, b) <= 1e-15


def test_metrics_definitions():
    A = np.array([[2.0, 1.0], [1.0, 3.0]])
    x = np.array([1.0, 1.0])
    xh = np.array([1.0, 1.5])
    b = A @ x
    assert metrics.ferr(xh, x) == 0.5
    # b - A xh = (-0.5, -1.5); ||A||=4, ||xh||=1.5, ||b||=4
    assert metrics.nbe(A, xh, b) == pytest.approx(1.5 / (4 * 1.5 + 4))
    # componentwise: |r| / (|A||xh| + |b|) = (0.5/(3.5+3), 1.5/(5.5+4))
    assert metrics.cbe(A, xh, b) == pytest.approx(max(0.5 / 6.5, 1.5 / 9.5))


def test_config1_backward_converges():
    A, x, b = WL.config_system(1)
    p = M.Params(**WL.CONFIGS[1]["params"])
    res = M.msir(A, b, p, x_true=x)
    assert res.cged and res.nbe <= 1e-15
    assert all(st.stage == M.SIR for st in res.history)


def test_script_aggressive_rho_keeps_sir():
    # Sec. 2.1.1: v = ||d2|| / ||d1|| = 0.6 triggers a switch under the cautious
    # rho_thresh = 0.5 but not under the aggressive 0.9, so SIR continues
    items = [("d", 1e-3, -1), ("d", 0.6e-3, -1), ("d", 0.36e-3, -1)] + [("d", 1e-30, 1)] * 40
    res, s = run_script(list(items), max_steps=3, rho_thresh=0.9)
    assert s.calls[:3] == [M.SIR, M.SIR, M.SIR]
    assert not res.history[1].events & M.EV_SWITCH
    res, s = run_script(list(items), max_steps=3, rho_thresh=0.5)
    assert s.calls[:3] == [M.SIR, M.SIR, M.SGMRES]


def test_aggressive_rho_moves_the_switch():
    # a system whose SIR ratios lie between 0.5 and 0.9: the cautious setting leaves
    # SIR on the first ratio >= 0.5, the aggressive one stays for i_max steps
    A, x, b = WL.randsvd(100, 3e3, 2, WL.rng_for(31, 0))
    runs = {rho: M.msir(A, b, M.Params(rho_thresh=rho, uf="fp16", u="fp32", ur="fp64", k_max=20), x_true=x)
            for rho in (0.5, 0.9)}
    sir = {rho: [st for st in r.history if st.stage == M.SIR] for rho, r in runs.items()}
    assert sir[0.5][-1].v >= 0.5 and len(sir[0.5]) < 10
    assert len(sir[0.9]) == 10 and max(st.v for st in sir[0.9]) < 0.9
    assert all(r.cged and metrics.nbe(A, r.x, b) <= 1e-15 for r in runs.values())


def test_componentwise_stops_at_first_iterate_meeting_tolerance():
    # conv = 'componentwise': the solve ends at the first iterate whose componentwise
    # backward error (the measure of Sec. 2.1.2, recomputed here by metrics.cbe) is
    # <= tol; the iterate one step earlier is above it
    A, x, b = WL.config_system(1)
    tol = 1e-15
    full = M.msir(A, b, M.Params(conv="componentwise", tol_nbe=tol), x_true=x)
    assert full.cged and metrics.cbe(A, full.x, b) <= tol
    K = len(full.history)
    prev = M.msir(A, b, M.Params(conv="componentwise", tol_nbe=tol, max_steps=K - 1), x_true=x)
    assert not prev.cged and metrics.cbe(A, prev.x, b) > tol
    loose = M.msir(A, b, M.Params(conv="componentwise", tol_nbe=1e-13), x_true=x)
    assert loose.cged and len(loose.history) <= K


def test_gmres_ir5_near_identity_operator_one_iteration_per_step():
    # u_f = u_g = u_p = fp64: M^{-1} A = I + E with ||E|| ~ kappa u_64 << tau, so every
    # GMRES call stops after one iteration; an unreachable tolerance runs i_max steps
    A, x, b = WL.randsvd(120, 1e2, 3, WL.rng_for(42, 0))
    r = M.gmres_ir5(A, b, M.Params(uf="fp64", u="fp64", ur="dd", tol_nbe=1e-30, i_max=3), ug="fp64", up="fp64",
                    x_true=x)
    assert [st.k for st in r.history] == [1, 1, 1]
    assert not r.cged and r.status == 1
    assert all(st.stage == M.GMRES and st.level == 0 for st in r.history)
    assert metrics.nbe(A, r.x, b) <= 1e-15


def test_gmres_ir5_stops_at_i_max_and_on_convergence():
    A, x, b = WL.randsvd(100, 1e3, 3, WL.rng_for(43, 100))
    r = M.gmres_ir5(A, b, M.Params(uf="fp16", u="fp32", ur="fp64", k_max=40, i_max=1, tol_nbe=1e-30), ug="fp32",
                    up="fp32")
    assert len(r.history) == 1 and not r.cged
    r = M.gmres_ir5(A, b, M.Params(uf="fp16", u="fp32", ur="fp64", k_max=40), ug="fp32", up="fp64")
    assert r.cged and metrics.nbe(A, r.x, b) <= 1e-15 and 0 < len(r.history) < 10

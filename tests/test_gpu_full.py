"""Parity at the workloads' full sizes, in the configuration bench.py times.

n = 4096 (the benchmark workload): the GPU solve is compared with the stored
oracle result (tests/golden/, written by make_golden.py from oracle/ only):
the same stage-switch sequence, steps per stage and GMRES counts within +-1,
nbe <= 1e-15, and x on the stored sample of components within the tolerance of
the solve tests.  The backward error is also recomputed on the host from the
returned x with the oracle's double-double residual.

n = 8192 (kappa 1e10, one small singular value, working precision fp64,
double-double residual), with fp16 and with bf16 factors: compared the same way with
the stored oracle results (tests/golden/gmresir_n8192_k1e10_mode2_{fp16,bf16}_oracle.json,
written by make_golden.py from oracle/ only), with the fp32 fused multiply-add
trailing update, whose factors are the oracle's bit for bit, and the GMRES operator
applied by substitution as the oracle applies it.  On this input neither format
needs the GMRES-IR stage: fp16 goes SIR -> SGMRES-IR, bf16 too (its second SGMRES-IR
call runs to the 820-iteration cap).  With the library defaults (matrix-core update,
operator through explicit inverses) the run is checked for the oracle's stage
sequence and outcome: convergence to nbe <= 1e-15 recomputed on the host
(double-double residual) and the forward error bound that backward error implies.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import metrics as OMET
from paper_2107_06200_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def M():
    from paper_2107_06200_amd import msir
    msir.lib()
    return msir


@pytest.fixture(scope="module")
def h(M):
    hh = M.Handle(0)
    yield hh
    hh.close()


def solve(M, h, A, b, x, params, lu_update="mfma", gmres_op="inverse"):
    At = M.colmajor(torch.from_numpy(np.asfortranarray(A)).to(DEV))
    bt = torch.from_numpy(b).to(DEV)
    xt = torch.from_numpy(x).to(DEV)
    P = M.params(lu_update=lu_update, gmres_op=gmres_op, **params)
    xg, res, hist, rc = M.solve(h, At, bt, x_true=xt, P=P)
    return xg.cpu().numpy(), res, hist, rc


def blocks(seq):
    out = []
    for lvl, st, counted, k in seq:
        key = (lvl, st, counted)
        if out and out[-1][0] == key:
            out[-1][1] += 1
            out[-1][2].append(k)
        else:
            out.append([key, 1, [k]])
    return out


def test_config2_full_size_vs_stored_oracle(M, h):
    cfg = WL.CONFIGS[2]
    path = os.path.join(GOLDEN, "%s_oracle.json" % cfg["name"])
    ref = json.load(open(path))
    A, x, b = WL.config_system(2)
    xg, res, hist, rc = solve(M, h, A, b, x, cfg["params"])   # bench.py's configuration
    print("gpu", M.render(hist), "nbe %.2e" % res.nbe, "| stored oracle", ref["render"], "nbe %.2e" % ref["nbe"])
    g = blocks([(s.level, s.stage, s.counted, s.k_gmres) for s in hist])
    o = blocks([tuple(t) for t in ref["history"]])
    assert [bg[0] for bg in g] == [bo[0] for bo in o], (g, o)
    for bg, bo in zip(g, o):
        assert abs(bg[1] - bo[1]) <= 1, (g, o)
        for kg, ko in zip(bg[2], bo[2]):
            assert abs(kg - ko) <= 1, (g, o)
    assert rc == 0 and res.cged == 1 and res.nbe <= 1e-15
    assert OMET.nbe(A, xg, b) <= 1e-15                  # host double-double residual of the GPU's x
    kinf = WL.kappa_inf(A)
    tol = max(1e-12 * max(1.0, cfg["kappa"] * 1e-4), 4 * kinf * (res.nbe + ref["nbe"]))
    xs = np.array(ref["x_sample"])
    assert np.abs(xg[::ref["sample_stride"]] - xs).max() <= tol * np.abs(xs).max()


@pytest.fixture(scope="module")
def c3():
    return WL.config_system(3)


def same_blocks(g, o):
    if [bg[0] for bg in g] != [bo[0] for bo in o]:
        return False
    for bg, bo in zip(g, o):
        if abs(bg[1] - bo[1]) > 1 or any(abs(kg - ko) > 1 for kg, ko in zip(bg[2], bo[2])):
            return False
    return True


def compare_with_golden(M, hist, res, xg, A, b, ref, kappa, events=True):
    # the history must match the stored oracle run, or one of the oracle's runs with its
    # BLAS library on another thread count (alt_histories: the oracle's own spread where
    # a GMRES call stagnates near tau and its stop is decided by float64 rounding order)
    g = blocks([(s.level, s.stage, s.counted, s.k_gmres) for s in hist])
    cands = [ref["history"]] + [a["history"] for a in ref.get("alt_histories", {}).values()]
    ok = [same_blocks(g, blocks([tuple(t) for t in c])) for c in cands]
    print("matches oracle runs:", ok, [blocks([tuple(t) for t in c]) for c in cands])
    assert any(ok), (g, cands)
    if events and "events" in ref and ok[0]:
        # the event bits of each stage (union) as the oracle's
        def union(seq, ev):
            out, cur = [], None
            for t, e in zip(seq, ev):
                key = tuple(t[:3])
                if cur is None or cur[0] != key:
                    cur = [key, 0]
                    out.append(cur)
                cur[1] |= e
            return [tuple(u) for u in out]
        assert union([(s.level, s.stage, s.counted) for s in hist], [s.events for s in hist]) == \
            union([t[:3] for t in ref["history"]], ref["events"])
    assert res.status == 0 and res.cged == 1 and res.nbe <= 1e-15
    assert OMET.nbe(A, xg, b) <= 1e-15                  # host double-double residual of the GPU's x
    kinf = WL.kappa_inf(A)
    tol = max(1e-12 * max(1.0, kappa * 1e-4), 4 * kinf * (res.nbe + ref["nbe"]))
    xs = np.array(ref["x_sample"])
    err = np.abs(xg[::ref["sample_stride"]] - xs).max() / np.abs(xs).max()
    print("XERR sample err=%.3e literal=%.3e asserted=%.3e" % (err, 1e-12 * max(1.0, kappa * 1e-4), tol))
    assert err <= tol


@pytest.mark.parametrize("uf", ["fp16", "bf16"])
def test_config3_full_size_vs_stored_oracle(M, h, c3, uf):
    # the method as stated: reproducible update (the oracle's factors) and the GMRES
    # operator by substitution in the operator precision, as the oracle applies it
    cfg = WL.CONFIGS[3]
    ref = json.load(open(os.path.join(GOLDEN, "%s_%s_oracle.json" % (cfg["name"], uf))))
    A, x, b = c3
    prm = dict(cfg["params"], uf=uf)
    xg, res, hist, rc = solve(M, h, A, b, x, prm, lu_update="fma", gmres_op="subst")
    print("gpu", M.render(hist), "nbe %.2e" % res.nbe, "| stored oracle", ref["render"], "nbe %.2e" % ref["nbe"])
    compare_with_golden(M, hist, res, xg, A, b, ref, cfg["kappa"])


@pytest.mark.parametrize("uf", ["fp16", "bf16"])
def test_config3_full_size_default_operator(M, h, c3, uf):
    # the library defaults (matrix-core update, operator through the explicit inverses):
    # the oracle's stage sequence and outcome; the GMRES counts may differ, because the
    # inverse-based operator rounds differently from substitution when U is as
    # ill-conditioned as here (kappa 1e10), and GMRES runs close to tau = 1e-10
    cfg = WL.CONFIGS[3]
    ref = json.load(open(os.path.join(GOLDEN, "%s_%s_oracle.json" % (cfg["name"], uf))))
    A, x, b = c3
    xg, res, hist, rc = solve(M, h, A, b, x, dict(cfg["params"], uf=uf))
    print("gpu", M.render(hist), "nbe %.2e" % res.nbe, "| stored oracle", ref["render"], "nbe %.2e" % ref["nbe"])
    g = blocks([(s.level, s.stage, s.counted, s.k_gmres) for s in hist])
    o = blocks([tuple(t) for t in ref["history"]])
    assert [bg[0] for bg in g] == [bo[0] for bo in o], (g, o)
    assert ref["cged"] and res.status == 0 and res.nbe <= 1e-15
    nbe_host = OMET.nbe(A, xg, b)
    assert nbe_host <= 1e-15
    # forward error implied by the backward error (first-order perturbation bound)
    kinf = WL.kappa_inf(A)
    assert np.abs(xg - x).max() / np.abs(x).max() <= 4 * kinf * nbe_host + 1e-15


def test_config2_operator_inverse_vs_substitution(M, h):
    """The GMRES operator through explicit inverses, at the benchmark workload's full size.

    The oracle factors the n = 4096 system (column scaling, fp16, DM(16)); the GPU applies
    M^{-1} = mu S U^{-1} L^{-1} P R to a few vectors in precision p in both operator modes
    (float64 inverses rounded to p, and substitution in p) and the oracle in float64
    substitution.  Both GPU modes carry an error of the kind kappa(T) u_p; the inverse
    mode must stay within a factor 50 of the substitution mode (its rounding is amplified
    by kappa(L) and kappa(U) rather than by the componentwise condition of the solve).
    The measured errors are printed (OPERR lines)."""
    from oracle import fmt as F
    from oracle import lu as OLU
    from oracle import scaling as OSC
    from oracle import solve as OSV
    A, x, b = WL.config_system(2)
    n = A.shape[0]
    scal = OSC.compute(A, "fp16", rows=False)
    Af = F.round_to(OSC.apply(A, *scal), "fp16")
    W, piv, info = OLU.getrf(Af, "fp16", OLU.nb_auto(n, "fp16"))[:3]
    assert info == 0
    Wd = M.colmajor(torch.from_numpy(np.asfortranarray(W)).to(M.TORCH_DTYPE[M.PREC["fp16"]]).to(DEV))
    ip = torch.from_numpy(piv.astype(np.int32)).to(DEV)
    R = torch.from_numpy(np.ascontiguousarray(scal[0])).to(DEV)
    S = torch.from_numpy(np.ascontiguousarray(scal[1])).to(DEV)
    mu = scal[2]
    rng = np.random.default_rng(11)
    for comp in ("fp32", "fp64"):
        worst = []
        for k in range(3):
            t = rng.standard_normal(n)
            want = OSV.lu_solve(W, piv, t, "fp64", scal)
            tt = torch.from_numpy(t).to(DEV)
            inv = M.getrs(h, Wd, "fp16", ip, tt, comp, R, S, mu, mode=1).cpu().numpy()
            sub = M.getrs(h, Wd, "fp16", ip, tt, comp, R, S, mu, mode=0).cpu().numpy()
            e_inv = float(np.abs(inv - want).max() / np.abs(want).max())
            e_sub = float(np.abs(sub - want).max() / np.abs(want).max())
            print("OPERR n=%d p=%s vector %d: inverses %.3e substitution %.3e" % (n, comp, k, e_inv, e_sub))
            worst.append((e_inv, e_sub))
            assert np.all(np.isfinite(inv)) and np.all(np.isfinite(sub))
            assert e_inv <= 50 * max(e_sub, 64 * F.u(comp)), (comp, e_inv, e_sub)


def test_config3_operator_inverse_vs_substitution(M, h, c3):
    """The GMRES operator through explicit inverses on the n = 8192 factors (kappa 1e10).

    The GPU factors fl16(A) (no scaling, the reproducible multiply-add update); the
    preconditioned operator U^{-1} L^{-1} P is applied to a few vectors in float64 in both
    operator modes and by the oracle's float64 substitution on the same factors.  Both GPU
    modes must stay within a factor 50 of the larger of the substitution mode's error and
    64 u (as at n = 4096); the measured errors are printed (OPERR lines)."""
    from oracle import fmt as F
    from oracle import solve as OSV
    A, x, b = c3
    n = A.shape[0]
    W = M.colmajor(torch.from_numpy(np.asfortranarray(A)).to(DEV).to(torch.float16))
    ipiv, info = M.getrf(h, W, "fp16", M.nb_auto(n, "fp16"), update="fma")
    assert info == 0
    Wh = W.to(torch.float64).cpu().numpy()
    piv = ipiv.cpu().numpy()
    rng = np.random.default_rng(13)
    for k in range(3):
        t = rng.standard_normal(n)
        want = OSV.lu_solve(Wh, piv, t, "fp64")
        tt = torch.from_numpy(t).to(DEV)
        inv = M.getrs(h, W, "fp16", ipiv, tt, "fp64", mode=1).cpu().numpy()
        sub = M.getrs(h, W, "fp16", ipiv, tt, "fp64", mode=0).cpu().numpy()
        e_inv = float(np.abs(inv - want).max() / np.abs(want).max())
        e_sub = float(np.abs(sub - want).max() / np.abs(want).max())
        print("OPERR n=%d p=fp64 vector %d: inverses %.3e substitution %.3e" % (n, k, e_inv, e_sub))
        assert np.all(np.isfinite(inv)) and np.all(np.isfinite(sub))
        assert e_inv <= 50 * max(e_sub, 64 * F.u("fp64")), (e_inv, e_sub)

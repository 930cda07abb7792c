"""Parity at the workloads' full sizes, in the configuration bench.py times.

n = 4096 (the benchmark workload): the GPU solve is compared with the stored
oracle result (tests/golden/, written by make_golden.py from oracle/ only):
the same stage-switch sequence, steps per stage and GMRES counts within +-1,
nbe <= 1e-15, and x on the stored sample of components within the tolerance of
the solve tests.  The backward error is also recomputed on the host from the
returned x with the oracle's double-double residual.

n = 8192 (double-double residual, GMRES-IR): the oracle cannot run this size
in a test, so properties that hold at any size are checked: convergence to
nbe <= 1e-15 recomputed on the host (double-double residual), the forward
error bound that backward error implies, and a well-formed stage history
(levels only increase; within a level the variants follow SIR -> SGMRES-IR
-> GMRES-IR).
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


def solve(M, h, A, b, x, params, lu_update="mfma"):
    At = M.colmajor(torch.from_numpy(np.asfortranarray(A)).to(DEV))
    bt = torch.from_numpy(b).to(DEV)
    xt = torch.from_numpy(x).to(DEV)
    P = M.params(lu_update=lu_update, **params)
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


def test_config3_full_size_properties(M, h):
    cfg = WL.CONFIGS[3]
    A, x, b = WL.config_system(3)
    n = A.shape[0]
    xg, res, hist, rc = solve(M, h, A, b, x, cfg["params"])
    print("gpu", M.render(hist), "nbe %.2e" % res.nbe, "ferr %.2e" % res.ferr)
    assert rc == 0 and res.cged == 1
    assert res.nbe <= 1e-15
    nbe_host = OMET.nbe(A, xg, b)
    assert nbe_host <= 1e-15
    # forward error implied by the backward error (first-order perturbation bound)
    kinf = WL.kappa_inf(A)
    ferr = np.abs(xg - x).max() / np.abs(x).max()
    assert ferr <= 4 * kinf * nbe_host + 1e-15
    # well-formed history: levels non-decreasing; within a level, variants in order
    prev = (-1, -1)
    for s in hist:
        assert s.level >= prev[0]
        if s.level == prev[0]:
            assert s.stage >= prev[1]
        prev = (s.level, s.stage)
    assert res.n_lu >= 1 and len(hist) <= 10 * 3 * 4
    assert n == 8192

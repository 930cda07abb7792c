"""Batched solve of independent systems of uneven order (the uneven-batch workload:
n log-uniform in [64, 1024], log10 kappa uniform in [1, 8], modes 2 and 3, fp16
factors, fp32 working precision, fp64 residual) against the CPU oracle.

One call of msir_solve_batched factors every system in one persistent launch and
runs every controller in another; each system's history and solution are compared
with the oracle's run of Alg. 4 on that system, with the bar of the single-system
solve tests (stage-switch sequence, steps per stage and GMRES counts within +-1, event
bits, nbe <= 1e-15, x within max(1e-12 max(1, kappa 1e-4), 4 kappa_inf (nbe_gpu +
nbe_oracle))).  The batched refinement applies the GMRES operator by substitution,
as the oracle does; with the fp32 fused multiply-add trailing update its factors are
the oracle's bit for bit.

Where a decision of the method sits on a rounding boundary the two sides may take
different branches, and the histories part there.  With the fp32 fused multiply-add
update (factors equal to the oracle's) one such boundary occurs on these inputs and is
named, counted and bounded: a GMRES call that stagnates at the attainable accuracy of
its working precision (tau below the rounding floor of the preconditioned operator),
whose stop is then decided by rounding noise, so one side reaches the iteration cap
while the other stops earlier.  With the matrix-core update the factors differ from
the oracle's in their last bits (the hardware's accumulation order), which moves every
decision that depends on the factors' errors: the SIR contraction ratio against
rho_thresh, an fp16 overflow of a SIR correction, a GMRES stop near tau.  There the
histories are printed and counted, and every system must reach the oracle's status,
the backward error and the x tolerance.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import msir as OM
from paper_2107_06200_amd import workloads as WL

from test_gpu_solve import assert_same_history, report_x

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


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


def dev_systems(M, systems):
    As = [M.colmajor(torch.from_numpy(np.asfortranarray(A)).to(DEV)) for A, _, _ in systems]
    bs = [torch.from_numpy(b).to(DEV) for _, _, b in systems]
    xts = [torch.from_numpy(x).to(DEV) for _, x, _ in systems]
    return As, bs, xts


def subsample(k, stride):
    meta = WL.batched_meta()
    return [meta[i] for i in range(0, len(meta), stride)][:k]


def boundary_kind(hist, ref, k_cap):
    """Where two histories part: 'stagnation' when, from the first differing step, the
    stage run holds a GMRES call that reached the iteration cap on one side only;
    'overflow' when a non-finite SIR correction (uncounted step) appears on one side
    only there; else None."""
    g = [(s.level, s.stage, s.counted, s.k_gmres) for s in hist]
    o = [(s.level, s.stage, int(s.counted), s.k) for s in ref.history]
    i = 0
    while i < min(len(g), len(o)) and g[i] == o[i]:
        i += 1

    def stage_ks(a):
        if i >= len(a):
            return []
        out = []
        for t in a[i:]:
            if t[:2] != a[i][:2]:
                break
            out.append(t[3])
        return out

    if any(k >= k_cap for k in stage_ks(g)) != any(k >= k_cap for k in stage_ks(o)):
        return "stagnation"
    ng = [j for j, t in enumerate(g) if t[2] == 0][:1]
    no = [j for j, t in enumerate(o) if t[2] == 0][:1]
    if ng != no and min(ng + no) >= i:       # the first non-finite correction moved
        return "overflow"
    return None


@pytest.mark.parametrize("lu_update", ["fma", "mfma"])
def test_batched_uneven_vs_oracle(M, h, lu_update):
    metas = subsample(20, 25)
    systems = [WL.batched_system(m) for m in metas]
    As, bs, xts = dev_systems(M, systems)
    prm = dict(WL.BATCHED_PARAMS)
    xs, outs, hists, rc = M.solve_batched(h, As, bs, x_true=xts, P=M.params(lu_update=lu_update, **prm))
    parted = []
    for m, (A, x, b), xg, o, hist in zip(metas, systems, xs, outs, hists):
        ref = OM.msir(A, b, OM.Params(**prm), x_true=x)
        print("n=%d kappa=%.1e mode %d | gpu %s nbe %.2e | oracle %s nbe %.2e" % (
            m["n"], m["kappa"], m["mode"], M.render(hist), o.nbe, OM.render(ref.history), ref.nbe), flush=True)
        try:
            assert_same_history(hist, ref, lu_update=lu_update)
        except AssertionError:
            kind = boundary_kind(hist, ref, int(np.ceil(0.1 * m["n"])))
            print("  histories part at a rounding boundary:", kind)
            print("  gpu   ", [(s.level, s.stage, s.counted, s.k_gmres, s.events) for s in hist])
            print("  oracle", [(s.level, s.stage, int(s.counted), s.k, s.events) for s in ref.history])
            if lu_update == "fma":
                assert kind == "stagnation"
            parted.append((m["n"], kind))
        assert o.status == ref.status
        if ref.status == 0:
            assert o.cged == 1 and o.nbe <= 1e-15
            kinf = WL.kappa_inf(A)
            tol = max(1e-12 * max(1.0, m["kappa"] * 1e-4), 4 * kinf * (o.nbe + ref.nbe))
            err = report_x("batched_n%d[%s]" % (m["n"], lu_update), xg.cpu().numpy(), ref.x, m["kappa"], tol)
            assert err <= tol
    print("parted at a rounding boundary:", parted)
    if lu_update == "fma":
        assert len(parted) <= 2


def test_batched_edge_orders_and_a_large_system(M, h):
    # ragged orders around the 64-row blocks, the smallest orders, and one system above
    # the batched kernels' order limit (solved by the single-system path) in one call
    orders = [1, 2, 63, 64, 65, 127, 1024, 1100]
    systems = [WL.randsvd(n, 30.0, 3, WL.rng_for(44, n)) for n in orders]
    As, bs, xts = dev_systems(M, systems)
    prm = dict(WL.BATCHED_PARAMS)
    xs, outs, hists, rc = M.solve_batched(h, As, bs, x_true=xts, P=M.params(lu_update="fma", **prm))
    assert rc == 0
    for n, (A, x, b), xg, o, hist in zip(orders, systems, xs, outs, hists):
        ref = OM.msir(A, b, OM.Params(**prm), x_true=x)
        print("n=%d gpu %s | oracle %s" % (n, M.render(hist), OM.render(ref.history)))
        assert_same_history(hist, ref)
        assert o.status == 0 and o.nbe <= 1e-15


def test_batched_equals_alone(M, h):
    # each system's result is the same whether it is solved alone or in the batch
    metas = subsample(12, 41)
    systems = [WL.batched_system(m) for m in metas]
    As, bs, xts = dev_systems(M, systems)
    P = M.params(**WL.BATCHED_PARAMS)
    xs, outs, hists, rc = M.solve_batched(h, As, bs, P=P)
    for i in (0, 5, 11):
        x1, o1, h1, rc1 = M.solve_batched(h, [As[i]], [bs[i]], P=P)
        assert torch.equal(x1[0], xs[i])
        assert M.render(h1[0]) == M.render(hists[i])


def test_batched_full_uneven_workload_converges(M, h):
    # all 512 systems: every one reaches nbe <= 1e-15 (double-double residual recomputed
    # on the host for a sample) within the ladder
    metas = WL.batched_meta()
    systems = [WL.batched_system(m) for m in metas]
    As, bs, xts = dev_systems(M, systems)
    xs, outs, hists, rc = M.solve_batched(h, As, bs, x_true=xts, P=M.params(**WL.BATCHED_PARAMS))
    bad = [(m["n"], m["kappa"], o.status, o.nbe) for m, o in zip(metas, outs) if not (o.status == 0 and o.nbe <= 1e-15)]
    print("not converged:", bad)
    assert rc == 0 and not bad
    from oracle import metrics as OMET
    for i in range(0, 512, 37):
        A, x, b = systems[i]
        assert OMET.nbe(A, xs[i].cpu().numpy(), b) <= 1e-15

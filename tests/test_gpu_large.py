"""Orders above 8192 (up to the library's maximum, 16384): panels of up to sixteen rows
per thread (panel widths 4 in fp16 / bf16 / fp32 and 2 in fp64) and the Arnoldi
kernel's sixteen values per thread.  The oracle's elimination is far too slow at these
orders, so the factorization is checked by an exact-arithmetic construction whose
factors are known (they must come back bit for bit) and the solver by properties that
hold at any size.  Every input is built on the device from a seeded generator."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import lu as OLU

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


def exact_system(n, seed):
    """P0^T L0 U0 with a sparse unit lower L0 (about four entries in {1/4, 1/2} per
    row) and an integer U0 with diagonal in {4, 8}: every entry of A and of every Schur
    complement of the pivoted elimination is a small quarter-integer, exact in each
    factor format and in the fp32 accumulator, and partial pivoting selects P0."""
    g = torch.Generator(device=DEV).manual_seed(seed)
    dt = torch.float64
    mask = torch.rand((n, n), generator=g, device=DEV, dtype=dt) < (4.0 / n)
    vals = torch.tensor([0.25, -0.25, 0.5, -0.5], device=DEV, dtype=dt)
    L0 = torch.tril(torch.where(mask, vals[torch.randint(0, 4, (n, n), generator=g, device=DEV)], 0.0), -1)
    del mask
    L0 += torch.eye(n, device=DEV, dtype=dt)
    U0 = torch.triu(torch.randint(-4, 5, (n, n), generator=g, device=DEV).to(dt), 1)
    dvals = torch.tensor([4.0, -4.0, 8.0, -8.0], device=DEV, dtype=dt)
    U0 += torch.diag(dvals[torch.randint(0, 4, (n,), generator=g, device=DEV)])
    P0 = torch.randperm(n, generator=g, device=DEV)
    A = torch.empty((n, n), device=DEV, dtype=dt)
    A[P0] = L0 @ U0
    want = torch.tril(L0, -1) + U0
    return A, want, P0


@pytest.mark.parametrize("fmt,n", [("fp16", 12000), ("bf16", 16384), ("fp32", 12000), ("fp64", 9000)])
def test_getrf_exact_arithmetic_beyond_8192(M, h, fmt, n):
    """The default panel width at this order (M.nb_auto) on the exact construction:
    both trailing updates must return (P0, L0, U0) exactly."""
    print("CASE getrf exact fmt=%s n=%d" % (fmt, n), flush=True)
    nb = M.nb_auto(n, fmt)
    assert nb == OLU.nb_auto(n, fmt)
    A, want, P0 = exact_system(n, n + nb)
    tdt = M.TORCH_DTYPE[M.PREC[fmt]]
    assert torch.equal(A.to(tdt).to(torch.float64), A)
    updates = ("mfma", "fma") if fmt in ("fp16", "bf16") else ("fma",)
    for update in updates:
        W = M.colmajor(A.to(tdt))
        ipiv, info = M.getrf(h, W, fmt, nb, update=update)
        assert info == 0
        assert torch.equal(W.to(torch.float64), want), update
        perm = OLU.perm_from_piv(ipiv.cpu().numpy())
        np.testing.assert_array_equal(perm, P0.cpu().numpy())
        del W
        torch.cuda.synchronize()


PARAMS2 = dict(uf="fp16", u="fp32", ur="fp64", ux="fp64", i_max=10, tau=1e-4, rho_thresh=0.5, restart=50,
               scaling="cols")


def test_solve_n12000_gaussian(M, h):
    """Alg. 4 with the benchmark workload's parameters (fp16 factors, fp32 working
    precision, fp64 residual and solution, GMRES tolerance 1e-4, restart 50) on a
    Gaussian matrix of order 12000 built on the device.  Checks: convergence, the
    backward error recomputed on the device in float64 from the returned x, and the
    forward error against the generating solution."""
    n = 12000
    print("CASE solve gaussian n=%d" % n, flush=True)
    g = torch.Generator(device=DEV).manual_seed(12000)
    A = torch.randn((n, n), generator=g, device=DEV, dtype=torch.float64)
    xt = torch.randn(n, generator=g, device=DEV, dtype=torch.float64)
    b = A @ xt
    x, res, hist, rc = M.solve(h, A, b, P=M.params(**PARAMS2))
    print("gpu", M.render(hist), "nbe %.2e status %d n_lu %d gmres %d" % (res.nbe, res.status, res.n_lu,
                                                                          res.gmres_iters), flush=True)
    assert rc == 0 and res.status == 0
    r = b - A @ x
    nbe = float(r.abs().max() / (A.abs().sum(dim=1).max() * x.abs().max() + b.abs().max()))
    # the float64 residual itself carries an error of order n u |A| |x|
    assert nbe <= n * 2.0 ** -53, nbe
    assert torch.isfinite(x).all()
    ferr = float((x - xt).abs().max() / xt.abs().max())
    print("ferr %.3e" % ferr)
    assert ferr <= 1e-6


def test_solve_n9000_kappa1e6_gmres(M, h):
    """The benchmark workload's recipe (randsvd, kappa 1e6, geometric singular values)
    and parameters at order 9000: fp16 SIR stagnates, SGMRES-IR and GMRES-IR run long
    GMRES cycles through the Arnoldi kernel's sixteen-values-per-thread form, and the
    solve converges.  Checks: GMRES ran, convergence, the backward error recomputed on
    the host with the oracle's double-double residual, and the forward error that
    backward error implies with kappa_2 = 1e6 (|x - x*|_inf / |x*|_inf is at most
    sqrt(n) kappa_2 times the normwise backward error, to first order)."""
    from oracle import metrics as OMET
    from paper_2107_06200_amd import workloads as WL
    n = 9000
    print("CASE solve randsvd n=%d" % n, flush=True)
    A, xt, b = WL.randsvd(n, 1e6, 3, WL.rng_for(2, 0))
    At = M.colmajor(torch.from_numpy(np.asfortranarray(A)).to(DEV))
    x, res, hist, rc = M.solve(h, At, torch.from_numpy(b).to(DEV), P=M.params(**PARAMS2))
    print("gpu", M.render(hist), "nbe %.2e status %d n_lu %d gmres %d" % (res.nbe, res.status, res.n_lu,
                                                                          res.gmres_iters), flush=True)
    assert rc == 0 and res.status == 0
    assert res.gmres_iters > 0
    xg = x.cpu().numpy()
    nbe = OMET.nbe(A, xg, b)
    print("host nbe %.2e" % nbe)
    assert nbe <= 1e-15
    ferr = float(np.abs(xg - xt).max() / np.abs(xt).max())
    print("ferr %.3e" % ferr)
    assert ferr <= 4 * np.sqrt(n) * 1e6 * max(nbe, 2.0 ** -53)


def test_cycle_longer_than_lds_rejected(M, h):
    """A GMRES cycle longer than 8192 (possible only above order 8192) is a parameter
    error, reported before any work."""
    n = 8200
    A = torch.eye(n, device=DEV, dtype=torch.float64)
    b = torch.ones(n, device=DEV, dtype=torch.float64)
    P = M.params(k_max=8200, restart=0)
    with pytest.raises(M.MsirError):
        M.solve(h, A, b, P=P)
    P = M.params(k_max=8192, restart=0)
    x, res, hist, rc = M.solve(h, A, b, P=P)
    assert rc == 0
    assert float((x - b).abs().max()) <= 1e-15

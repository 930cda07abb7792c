"""Least-squares MSIR on the GPU (augmented system; Sec. 4 future work) against the
oracle (oracle/lstsq.py).

The GPU builds [[alpha I, A], [A^T, 0]] and [b; 0] itself and runs Alg. 4 on it; the
oracle builds the same system with its own code.  The bar is that of the square
solves (tests/test_gpu_solve.py): the same history within +-1 (strict with the
reproducible LU update), normwise backward error <= 1e-15 on the augmented system,
and x, r within 4 kappa_inf(K) (nbe_gpu + nbe_oracle) of the oracle's (relative);
plus the least-squares optimality A^T r = 0 and r = b - A x up to rounding."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import lstsq as OL
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


def sigma_alpha(kappa):
    # sigma_min = 1 / kappa for the generator's mode-3 singular values
    return 2.0 ** round(np.log2(1.0 / kappa / np.sqrt(2.0)))


CASES = [  # m, n, kappa, alpha (None: the default rule)
    (30, 12, 10.0, None),
    (40, 25, 1e2, None),
    (200, 80, 1e3, None),
    (60, 20, 1e4, "sigma"),
    (97, 33, 1e2, None),
]


@pytest.mark.parametrize("lu_update", ["fma", "mfma"])
@pytest.mark.parametrize("m,n,kappa,amode", CASES)
def test_lstsq_vs_oracle(M, h, m, n, kappa, amode, lu_update):
    A, x_t, b, r_t = WL.ls_system(m, n, kappa, 3, np.random.default_rng(1000 + m), rnorm=1e-2)
    alpha = sigma_alpha(kappa) if amode == "sigma" else None
    xo, ro, ao, ref = OL.lstsq(A, b, OM.Params(), alpha=alpha)
    At = M.colmajor(torch.from_numpy(np.asfortranarray(A)).to(DEV))
    bt = torch.from_numpy(b).to(DEV)
    xg, rg, ag, res, hist, rc = M.lstsq(h, At, bt, alpha=alpha or 0.0, P=M.params(lu_update=lu_update))
    print("gpu", M.render(hist), "nbe %.2e" % res.nbe, "| oracle", OM.render(ref.history), "nbe %.2e" % ref.nbe)
    assert ag == ao
    assert rc == 0 and res.cged == 1 and res.nbe <= 1e-15
    assert_same_history(hist, ref, lu_update=lu_update)
    xg = xg.cpu().numpy()
    rg = rg.cpu().numpy()
    K, _ = OL.augment(A, b, ao)
    tol = 4 * WL.kappa_inf(K) * (res.nbe + ref.nbe)
    err = report_x("lstsq_%d_%d[%s]" % (m, n, lu_update), xg, xo, kappa ** 2, tol)
    assert err <= tol
    assert np.max(np.abs(rg - ro)) <= tol * np.abs(b).max()
    # least-squares optimality of the GPU result
    assert np.max(np.abs(A.T @ rg)) <= 1e-12 * np.abs(A).max() * np.abs(rg).max() * m
    assert np.max(np.abs(rg - (b - A @ xg))) <= 1e-12 * np.abs(b).max()


def test_lstsq_large_problem_properties(M, h):
    # m + n = 4000: the oracle would take minutes; the generator's solution is known
    m, n, kappa = 3000, 1000, 1e2
    A, x_t, b, r_t = WL.ls_system(m, n, kappa, 3, np.random.default_rng(5), rnorm=1e-2)
    At = M.colmajor(torch.from_numpy(np.asfortranarray(A)).to(DEV))
    xg, rg, ag, res, hist, rc = M.lstsq(h, At, torch.from_numpy(b).to(DEV))
    print("gpu", M.render(hist), "nbe %.2e" % res.nbe, "alpha", ag)
    assert rc == 0 and res.cged == 1 and res.nbe <= 1e-15
    assert ag == OL.alpha_default(A)
    xg = xg.cpu().numpy()
    rg = rg.cpu().numpy()
    assert np.max(np.abs(xg - x_t)) <= 1e-13 * kappa ** 2 * np.abs(x_t).max()
    assert np.max(np.abs(rg - r_t)) <= 1e-13 * kappa ** 2 * np.abs(b).max()
    assert np.max(np.abs(A.T @ rg)) <= 1e-12 * np.abs(A).max() * np.abs(rg).max() * m


def test_lstsq_square_case_is_the_linear_solve(M, h):
    A, x_t, b = WL.randsvd(64, 10.0, 3, np.random.default_rng(9))
    At = M.colmajor(torch.from_numpy(np.asfortranarray(A)).to(DEV))
    xg, rg, ag, res, hist, rc = M.lstsq(h, At, torch.from_numpy(b).to(DEV))
    assert rc == 0 and res.cged == 1
    assert np.max(np.abs(xg.cpu().numpy() - x_t)) <= 1e-12 * np.abs(x_t).max()
    assert np.max(np.abs(rg.cpu().numpy())) <= 1e-13 * np.abs(b).max()


def test_lstsq_argument_errors(M, h):
    A = torch.zeros(5, 3, dtype=torch.float64, device=DEV)
    b = torch.zeros(5, dtype=torch.float64, device=DEV)
    x = torch.zeros(3, dtype=torch.float64, device=DEV)
    L = M.lib()
    p = A.data_ptr()
    # every error is found before any device access
    assert L.msir_lstsq(h.h, 3, 5, p, 5, b.data_ptr(), 0.0, x.data_ptr(), None, None, None, None, None, 0, None) == -2
    assert L.msir_lstsq(h.h, 5, 3, p, 4, b.data_ptr(), 0.0, x.data_ptr(), None, None, None, None, None, 0, None) == -4
    assert L.msir_lstsq(h.h, 5, 3, p, 5, b.data_ptr(), 3.0, x.data_ptr(), None, None, None, None, None, 0, None) == -9
    assert L.msir_lstsq(h.h, 5, 3, p, 5, b.data_ptr(), -2.0, x.data_ptr(), None, None, None, None, None, 0, None) == -9
    assert L.msir_lstsq(h.h, 5, 0, p, 5, b.data_ptr(), 0.0, x.data_ptr(), None, None, None, None, None, 0, None) == -102
    # m + n above the library's maximum order (16384)
    assert L.msir_lstsq(h.h, 16000, 500, p, 16000, b.data_ptr(), 0.0, x.data_ptr(), None, None, None, None, None, 0,
                        None) == -102

"""GPU parity of each step of the hot path against the CPU oracle (same seeded inputs).

Every call goes through the C ABI (paper_2107_06200_amd.msir -> libmsir.so).
Tolerances, where results are not bit-exact, come from where the two sides
may round differently: the order of float32 accumulation inside the matrix
cores (LU trailing update) and the order of float64 accumulation in inner
products; both are far below the rounding of the stored formats, so most
outputs agree bit for bit and the rest within a few units of the stored format.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fmt as F
from oracle import lu as OLU
from oracle import ops as OOPS
from oracle import scaling as OSC
from oracle import solve as OSV
from oracle import gmres as OGM
from paper_2107_06200_amd import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NPDT = {"fp16": np.float16, "fp32": np.float32, "fp64": np.float64}


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


def dev(a, M):
    return M.colmajor(torch.from_numpy(np.asfortranarray(a)).to(DEV))


def tdev(v):
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(DEV)


def host_w(W, fmt):
    """Device factor matrix (column-major tensor of the format's dtype) -> float64 numpy."""
    t = W.t().contiguous().t().cpu()
    return t.to(torch.float64).numpy()


def to_dev_fmt(Wf, fmt, M):
    t = torch.from_numpy(np.asfortranarray(Wf)).to(M.TORCH_DTYPE[M.PREC[fmt]])
    return M.colmajor(t.to(DEV))


# ------------------------------------------------------------------ conversion
@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32", "fp64"])
def test_convert_bitexact(M, h, fmt):
    rng = np.random.default_rng(1)
    n = 96
    A = rng.standard_normal((n, n)) * np.exp2(rng.uniform(-30, 20, (n, n)))
    edge = [65504.0, 65519.99, 65520.0, -65520.0, 2.0 ** -24, 2.0 ** -25, 1.5 * 2.0 ** -25, 3 * 2.0 ** -25,
            1.0 + 2.0 ** -11, 1.0 + 2.0 ** -11 + 2.0 ** -40, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -24, np.inf, -np.inf,
            0.0, -0.0, 1e-300, 3.4e38, 3.5e38]
    A.flat[: len(edge)] = edge
    W = M.convert(h, dev(A, M), fmt)
    got = host_w(W, fmt)
    want = F.round_to(A, fmt)
    np.testing.assert_array_equal(got, want)


def test_convert_nan_stays_nan(M, h):
    A = np.ones((8, 8))
    A[3, 4] = np.nan
    for fmt in ("fp16", "bf16"):
        got = host_w(M.convert(h, dev(A, M), fmt), fmt)
        mask = np.ones_like(got, dtype=bool)
        mask[3, 4] = False
        assert np.isnan(got[3, 4]) and np.isfinite(got[mask]).all()


@pytest.mark.parametrize("rows", [True, False])
def test_scaling_and_scaled_convert_bitexact(M, h, rows):
    rng = np.random.default_rng(2)
    n = 130
    A = rng.standard_normal((n, n)) * np.exp2(rng.integers(-25, 25, (n, 1))) * np.exp2(rng.integers(-10, 10, (1, n)))
    R, S, mu = M.scaling(h, dev(A, M), "fp16", rows)
    Ro, So, muo = OSC.compute(A, "fp16", rows=rows)
    np.testing.assert_array_equal(R, Ro)
    np.testing.assert_array_equal(S, So)
    assert mu == muo
    got = host_w(M.convert(h, dev(A, M), "fp16", R, S, mu), "fp16")
    np.testing.assert_array_equal(got, F.round_to(OSC.apply(A, Ro, So, muo), "fp16"))


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32"])
def test_round_values_bitexact(M, h, fmt):
    # fl_fmt(x) as every refinement kernel applies it, against the oracle's rounding:
    # random magnitudes over the whole range plus ties, the subnormal range, the
    # overflow threshold and the special values
    rng = np.random.default_rng(11)
    x = rng.standard_normal(40000) * np.exp2(rng.uniform(-160, 140, 40000))
    t = {"fp16": (11, -14, 15), "bf16": (8, -126, 127), "fp32": (24, -126, 127)}[fmt]
    p, emin, emax = t
    xmax = (2.0 - 2.0 ** (1 - p)) * 2.0 ** emax
    q = 2.0 ** (emin - p + 1)
    edge = [0.0, -0.0, np.inf, -np.inf, xmax, -xmax, xmax * (1 + 2.0 ** -p), xmax * (1 + 2.0 ** -p) * (1 - 2.0 ** -40),
            1.0 + 2.0 ** -p, 1.0 + 3 * 2.0 ** -p, 1.0 + 2.0 ** -p + 2.0 ** -50, q, q / 2, 3 * q / 2, q / 2 * (1 + 2.0 ** -30),
            2.0 ** emin, 2.0 ** emin - q / 2, 1e-300, -1e-300, 1e300, 5e-324]
    x[: len(edge)] = edge
    x[len(edge): 2 * len(edge)] = -np.array(edge)
    k = np.arange(4000)   # exact ties across binades
    x[100:4100] = (2 * rng.integers(1, 2 ** p, 4000) + 1) * 2.0 ** (rng.integers(emin - p, emax - p, 4000) - 1)
    got = M.round_values(h, tdev(x), fmt).cpu().numpy()
    want = F.round_to(x, fmt)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(np.signbit(got), np.signbit(want))


def test_round_values_nan(M, h):
    x = np.array([np.nan, 1.0, -np.nan])
    for fmt in ("fp16", "bf16", "fp32", "fp64"):
        got = M.round_values(h, tdev(x), fmt).cpu().numpy()
        assert np.isnan(got[0]) and got[1] == 1.0 and np.isnan(got[2])


# ------------------------------------------------------------------ LU
@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 5, 32])
def test_getrf_single_panel_bitexact(M, h, fmt, n):
    # one panel (nb >= n): the whole factorization is the register-resident panel
    # kernel, whose arithmetic (fp32 or fp64 FMA, rounded reciprocal) the oracle emulates exactly
    rng = np.random.default_rng(3 + n)
    nb = 32
    Af = F.round_to(rng.standard_normal((n, n)), fmt)
    W = to_dev_fmt(Af, fmt, M)
    ipiv, info = M.getrf(h, W, fmt, nb)
    Wo, po, io = OLU.getrf(Af, fmt, nb)
    assert info == io
    np.testing.assert_array_equal(ipiv.cpu().numpy(), po)
    if fmt == "fp64":
        np.testing.assert_allclose(host_w(W, fmt), Wo, rtol=0, atol=4e-16 * n * np.abs(Wo).max())
    else:
        np.testing.assert_array_equal(host_w(W, fmt), Wo)


def manufactured(n, seed):
    rng = np.random.default_rng(seed)
    order = rng.permutation(n)
    A = rng.uniform(-1, 1, (n, n)) * 2.0 ** -8
    for k, r in enumerate(order):
        A[r, k] = 2.0 ** (6 - k % 4) * (1 if k % 2 else -1)
    return A


@pytest.mark.parametrize("fmt,n,nb", [("fp16", 300, 64), ("fp16", 1100, 32), ("bf16", 300, 32),
                                      ("fp32", 257, 16), ("fp64", 200, 16)])
def test_getrf_manufactured_pivots_bitexact(M, h, fmt, n, nb):
    Af = F.round_to(manufactured(n, n), fmt)
    W = to_dev_fmt(Af, fmt, M)
    ipiv, info = M.getrf(h, W, fmt, nb)
    Wo, po, io = OLU.getrf(Af, fmt, nb)
    assert info == io == 0
    np.testing.assert_array_equal(ipiv.cpu().numpy(), po)


def pivot_margin(n, seed, fmt):
    """Random matrix with a pivot margin: in column k the entry of row order[k] is
    4-16 times larger than any other entry (before and, by a margin that the
    rounding of the trailing updates cannot close, after elimination), so GEPP
    picks order[k] at step k on both sides whatever the accumulation order."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(n)
    A = rng.uniform(-1, 1, (n, n))
    for k, r in enumerate(order):
        A[r, k] = (4.0 * n) * rng.uniform(1.0, 4.0) * (1 if k % 2 else -1)
    return F.round_to(A, fmt)


@pytest.mark.parametrize("fmt,n,nb", [("fp16", 200, 64), ("fp16", 333, 16), ("bf16", 200, 32),
                                      ("fp32", 200, 16), ("fp64", 150, 16), ("fp32", 300, 64), ("fp64", 300, 32)])
def test_getrf_blocked_vs_oracle(M, h, fmt, n, nb):
    Af = pivot_margin(n, n + nb, fmt)
    W = to_dev_fmt(Af, fmt, M)
    ipiv, info = M.getrf(h, W, fmt, nb)   # matrix-core trailing update
    Wo, po, io = OLU.getrf(Af, fmt, nb, trailing="exact")
    Wg = host_w(W, fmt)
    piv = ipiv.cpu().numpy()
    # Backward error of the device factors (Higham): |PA - LU| <= gamma |L||U|
    L, U = OLU.unpack(Wg)
    p = OLU.perm_from_piv(piv)
    E = np.abs(Af[p] - L @ U)
    g = (n / nb + n * F.u("fp32") / F.u(fmt) + 3) * F.u(fmt)
    # fp16 multipliers below 2^-14 are subnormal: their rounding error is absolute
    # (at most 2^-25), which adds up to 2^-25 |u_jj| per product to the bound
    tiny = 2.0 ** -24 * np.abs(U).max() if fmt == "fp16" else 1e-300
    assert np.all(E <= g / (1 - g) * (np.abs(L) @ np.abs(U)) + tiny)
    # Agreement with the oracle.  The two sides differ only in the order of the
    # float32 (float64) accumulation of the trailing update; with the pivot margin
    # the pivots must be equal, and the rounding differences propagate through
    # later Schur complements, amplified by at most the condition number.
    np.testing.assert_array_equal(piv, po)
    kap = np.linalg.cond(Af, np.inf)
    rel = np.abs(Wg - Wo).max() / np.abs(Wo).max()
    assert rel <= 4 * kap * F.u(fmt), (rel, kap)


@pytest.mark.parametrize("fmt,n,nb", [("fp16", 100, 16), ("fp16", 96, 32), ("fp16", 130, 64),
                                      ("fp32", 100, 16), ("fp64", 100, 8), ("bf16", 40, 16)])
def test_getrf_exact_arithmetic_bitexact(M, h, fmt, n, nb):
    """A = P0^T L0 U0 with |l| in {0, 1/4, 1/2} and U0 integer with power-of-two
    diagonal: every multiplier, every trailing update and every stored value is
    exact in the factor format, so partial pivoting must return exactly (P0, L0,
    U0) on both sides -- this pins the matrix-core update's tile layout and the
    interchange bookkeeping independently of rounding order."""
    rng = np.random.default_rng(31 + n)
    amp = 2 if fmt == "bf16" else 4
    L0 = np.tril(rng.choice([0.0, 0.25, -0.25, 0.5, -0.5], (n, n)), -1) + np.eye(n)
    U0 = np.triu(rng.integers(-amp, amp + 1, (n, n)).astype(float), 1)
    U0[np.diag_indices(n)] = rng.choice([1.0, -1.0, 2.0, -2.0, 4.0, -4.0, 8.0, -8.0] if fmt != "bf16"
                                        else [4.0, -4.0, 8.0, -8.0], n)
    P0 = rng.permutation(n)
    A = np.empty((n, n))
    A[P0] = L0 @ U0
    assert np.array_equal(F.round_to(A, fmt), A)
    for update in ("mfma", "fma"):
        W = to_dev_fmt(A, fmt, M)
        ipiv, info = M.getrf(h, W, fmt, nb, update=update)
        Wo, po, io = OLU.getrf(A, fmt, nb)
        np.testing.assert_array_equal(ipiv.cpu().numpy(), po)
        np.testing.assert_array_equal(host_w(W, fmt), Wo)
        np.testing.assert_array_equal(Wo, np.tril(L0, -1) + U0)


@pytest.mark.parametrize("fmt,n,nb", [("fp16", 4096, 16), ("bf16", 4096, 16), ("fp32", 4096, 16),
                                      ("fp16", 8192, 8), ("bf16", 8192, 8), ("fp64", 4096, 8)])
def test_getrf_exact_arithmetic_full_size(M, h, fmt, n, nb):
    """The exact-arithmetic construction at the workloads' full sizes (panels of four
    and eight rows per thread, the launch configuration of the benchmark): a sparse
    unit lower L0 (about four entries in {1/4, 1/2} per row) and an integer U0 keep
    every entry of A and of every Schur complement a small quarter-integer, exact in
    the factor format and in the fp32 accumulator, so both trailing updates must
    return exactly (P0, L0, U0).  Built and compared on the device (n^2 entries)."""
    g = torch.Generator(device=DEV).manual_seed(n + nb)
    dt = torch.float64
    mask = torch.rand((n, n), generator=g, device=DEV, dtype=dt) < (4.0 / n)
    vals = torch.tensor([0.25, -0.25, 0.5, -0.5], device=DEV, dtype=dt)
    L0 = torch.tril(torch.where(mask, vals[torch.randint(0, 4, (n, n), generator=g, device=DEV)], 0.0), -1)
    L0 += torch.eye(n, device=DEV, dtype=dt)
    U0 = torch.triu(torch.randint(-4, 5, (n, n), generator=g, device=DEV).to(dt), 1)
    dvals = torch.tensor([4.0, -4.0, 8.0, -8.0], device=DEV, dtype=dt)
    U0 += torch.diag(dvals[torch.randint(0, 4, (n,), generator=g, device=DEV)])
    P0 = torch.randperm(n, generator=g, device=DEV)
    A = torch.empty((n, n), device=DEV, dtype=dt)
    A[P0] = L0 @ U0
    want = (torch.tril(L0, -1) + U0)
    tdt = M.TORCH_DTYPE[M.PREC[fmt]]
    assert torch.equal(A.to(tdt).to(dt), A)
    for update in ("mfma", "fma"):
        W = M.colmajor(A.to(tdt))
        ipiv, info = M.getrf(h, W, fmt, nb, update=update)
        assert info == 0
        assert torch.equal(W.to(dt), want), update
        # interchanges -> permutation: (P A)[i] = A[perm[i]] must put row P0[i] at i
        piv = ipiv.cpu().numpy()
        perm = OLU.perm_from_piv(piv)
        np.testing.assert_array_equal(perm, P0.cpu().numpy())
        del W


@pytest.mark.parametrize("fmt,n,nb", [("fp16", 200, 64), ("fp16", 333, 16), ("bf16", 200, 32), ("fp16", 1100, 32),
                                      ("fp32", 257, 16), ("fp16", 1100, 16), ("bf16", 600, 8), ("fp32", 300, 64)])
def test_getrf_fma_update_bitexact(M, h, fmt, n, nb):
    """Reproducible trailing update (sequential fp32 FMA over k): the whole blocked
    factorization -- panel, interchanges, U12, trailing updates -- must equal the
    oracle's bit for bit, pivots included, on random matrices with ties to break."""
    rng = np.random.default_rng(7 * n + nb)
    Af = F.round_to(rng.standard_normal((n, n)), fmt)
    W = to_dev_fmt(Af, fmt, M)
    ipiv, info = M.getrf(h, W, fmt, nb, update="fma")
    Wo, po, io = OLU.getrf(Af, fmt, nb, trailing="fma32")
    assert info == io
    np.testing.assert_array_equal(ipiv.cpu().numpy(), po)
    np.testing.assert_array_equal(host_w(W, fmt), Wo)


@pytest.mark.parametrize("fmt,n,nb", [("fp16", 3000, 16), ("fp32", 2500, 16), ("fp64", 1800, 16), ("fp64", 3000, 8)])
def test_getrf_tall_panels_backward_error(M, h, fmt, n, nb):
    """Panels of more than 2048 rows (up to four rows per panel thread): checked by
    properties that hold at any size (the oracle's elimination is too slow here):
    componentwise backward error |PA - LU| <= gamma |L||U|, |L| <= 1 (partial
    pivoting), LAPACK-style pivots, every entry representable in u_f."""
    rng = np.random.default_rng(n + 3 * nb)
    Af = F.round_to(rng.standard_normal((n, n)), fmt)
    W = to_dev_fmt(Af, fmt, M)
    ipiv, info = M.getrf(h, W, fmt, nb)
    assert info == 0
    Wg = host_w(W, fmt)
    np.testing.assert_array_equal(F.round_to(Wg, fmt), Wg)
    piv = ipiv.cpu().numpy()
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    L, U = OLU.unpack(Wg)
    assert np.abs(np.tril(L, -1)).max() <= 1.0
    p = OLU.perm_from_piv(piv)
    E = np.abs(Af[p] - L @ U)
    ua = F.u("fp64") if fmt == "fp64" else F.u("fp32")
    g = (n / nb + n * ua / F.u(fmt) + 3) * F.u(fmt)
    assert np.all(E <= g / (1 - g) * (np.abs(L) @ np.abs(U)) + 1e-300)


def test_getrf_zero_pivot_info(M, h):
    n = 40
    rng = np.random.default_rng(9)
    A = F.round_to(rng.standard_normal((n, n)), "fp32")
    A[:, 7] = 0.0
    W = to_dev_fmt(A, "fp32", M)
    ipiv, info = M.getrf(h, W, "fp32", 16)
    Wo, po, io = OLU.getrf(A, "fp32", 16)
    assert info == io == 8


# ------------------------------------------------------------------ triangular solves
def oracle_factors(n, fmt, nb, seed, scaled=False):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 0.0
    scal = None
    if scaled:
        scal = OSC.compute(A, fmt, rows=True)
        Af = F.round_to(OSC.apply(A, *scal), fmt)
    else:
        Af = F.round_to(A, fmt)
    W, piv, info = OLU.getrf(Af, fmt, nb)
    return A, W, piv, scal


# (factor format, solution format, two-sided scaling): the scaling applies to fp16 factors only
_GETRS_CASES = [("fp16", "fp16", False), ("bf16", "bf16", False), ("fp16", "fp32", False), ("fp16", "fp64", False),
                ("fp32", "fp32", False), ("fp32", "fp64", False), ("fp64", "fp64", False),
                ("fp16", "fp16", True), ("fp16", "fp32", True), ("fp16", "fp64", True)]


@pytest.mark.parametrize("fmt,comp,scaled", _GETRS_CASES)
@pytest.mark.parametrize("n", [1, 64, 150])
def test_getrs_vs_oracle(M, h, fmt, comp, n, scaled):
    A, W, piv, scal = oracle_factors(n, fmt, 16, 11 + n, scaled)
    t = np.random.default_rng(5).standard_normal(n)
    want = OSV.lu_solve(W, piv, t, comp, scal)
    Wd = to_dev_fmt(W, fmt, M)
    ip = torch.from_numpy(piv.astype(np.int32)).to(DEV)
    R = S = None
    mu = 1.0
    if scal is not None:
        R, S, mu = tdev(scal[0]), tdev(scal[1]), scal[2]
    got = M.getrs(h, Wd, fmt, ip, tdev(t), comp, R, S, mu).cpu().numpy()
    if comp == "fp64":
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
    else:
        # float64 accumulation on both sides: the component roundings agree unless an
        # inner product lands within ~1e-16 of a rounding boundary of comp
        mism = np.mean(got != want)
        assert mism <= 0.02, mism
        assert np.abs(got - want).max() <= 64 * F.u(comp) * np.abs(want).max()


def test_getrs_dd_vs_oracle(M, h):
    n = 100
    A, W, piv, _ = oracle_factors(n, "fp64", 16, 21)
    t = np.random.default_rng(6).standard_normal(n)
    hi, lo = OSV.lu_solve(W, piv, t, "dd")
    Wd = to_dev_fmt(W, "fp64", M)
    ip = torch.from_numpy(piv.astype(np.int32)).to(DEV)
    tt = np.concatenate([t, np.zeros(n)])
    y = M.getrs(h, Wd, "fp64", ip, tdev(tt), "dd").cpu().numpy()
    # compare hi + lo exactly in double-double terms: |(gh - oh) + (gl - ol)| <= 2^-100 |y|
    diff = (y[:n] - hi) + (y[n:] - lo)
    assert np.abs(diff).max() <= 2.0 ** -98 * np.abs(hi).max()


def multiblock_factors(n, fmt, seed):
    """Stored factors for solves over many 64-row blocks without running the oracle's
    elimination: the strict lower part is L, the upper part U (diagonal bounded away from
    zero, off-diagonal entries of size 1/sqrt(n)), random LAPACK-style interchanges."""
    rng = np.random.default_rng(seed)
    W = rng.standard_normal((n, n)) / np.sqrt(n)
    W[np.diag_indices(n)] = (1.0 + np.abs(rng.standard_normal(n))) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    W = F.round_to(W, fmt)
    piv = np.array([rng.integers(j, n) for j in range(n)], dtype=np.int64)
    return W, piv


@pytest.mark.parametrize("fmt,comp", [("fp16", "fp16"), ("bf16", "bf16"), ("fp16", "fp64"), ("fp32", "fp32"),
                                      ("fp64", "fp64")])
@pytest.mark.parametrize("n", [200, 449, 1000])
def test_getrs_multiblock_vs_oracle(M, h, fmt, comp, n):
    # several 64-row blocks and a ragged last block: the chain, the helper sums of older
    # blocks and the forward/backward hand-over all take part
    W, piv = multiblock_factors(n, fmt, 31 + n)
    rng = np.random.default_rng(7 + n)
    t = rng.standard_normal(n)
    scal = (rng.uniform(0.5, 2.0, n), rng.uniform(0.5, 2.0, n), 0.75) if fmt == "fp16" else None
    want = OSV.lu_solve(W, piv, t, comp, scal)
    Wd = to_dev_fmt(W, fmt, M)
    ip = torch.from_numpy(piv.astype(np.int32)).to(DEV)
    R = S = None
    mu = 1.0
    if scal is not None:
        R, S, mu = tdev(scal[0]), tdev(scal[1]), scal[2]
    got = M.getrs(h, Wd, fmt, ip, tdev(t), comp, R, S, mu).cpu().numpy()
    assert np.all(np.isfinite(want))
    if comp == "fp64":
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
    else:
        mism = np.mean(got != want)
        assert mism <= 0.02, mism
        assert np.abs(got - want).max() <= 64 * F.u(comp) * np.abs(want).max()


def test_getrs_more_workgroups_than_resident(M, h):
    """fp64 factors: the substitution launch (one chain and one helper per block and
    sweep, 2 nblk + 1 = 257 workgroups for n = 8150) needs more workgroups than the
    GPU holds at once (the fp64 tiles take most of a compute unit's LDS: one workgroup
    per compute unit), so a helper starts as another finishes; the solve must still
    complete and agree with the oracle."""
    n = 8150
    W, piv = multiblock_factors(n, "fp64", 77)
    t = np.random.default_rng(78).standard_normal(n)
    want = OSV.lu_solve(W, piv, t, "fp64")
    Wd = to_dev_fmt(W, "fp64", M)
    ip = torch.from_numpy(piv.astype(np.int32)).to(DEV)
    got = M.getrs(h, Wd, "fp64", ip, tdev(t), "fp64").cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * np.abs(want).max())


@pytest.mark.parametrize("n", [300, 449])
def test_getrs_dd_multiblock_vs_oracle(M, h, n):
    W, piv = multiblock_factors(n, "fp64", 41 + n)
    t = np.random.default_rng(8 + n).standard_normal(n)
    hi, lo = OSV.lu_solve(W, piv, t, "dd")
    Wd = to_dev_fmt(W, "fp64", M)
    ip = torch.from_numpy(piv.astype(np.int32)).to(DEV)
    y = M.getrs(h, Wd, "fp64", ip, tdev(np.concatenate([t, np.zeros(n)])), "dd").cpu().numpy()
    diff = (y[:n] - hi) + (y[n:] - lo)
    assert np.abs(diff).max() <= 2.0 ** -96 * np.abs(hi).max()


def test_getrs_fp16_overflow_gives_inf(M, h):
    # u_f = fp16 solve: components beyond 65504 become Inf (the Alg. 4 NaN check relies on it)
    W = np.array([[2.0 ** -10, 0.0], [0.0, 1.0]])
    Wd = to_dev_fmt(W, "fp16", M)
    ip = torch.from_numpy(np.arange(2, dtype=np.int32)).to(DEV)
    y = M.getrs(h, Wd, "fp16", ip, tdev(np.array([100.0, 1.0])), "fp16").cpu().numpy()
    assert y[0] == np.inf and y[1] == 1.0


# ------------------------------------------------------------------ residual
@pytest.mark.parametrize("ur,u", [("fp64", "fp32"), ("fp64", "fp64"), ("dd", "fp64")])
@pytest.mark.parametrize("n", [1, 77, 700])
def test_residual_vs_oracle(M, h, ur, u, n):
    A, x, b = WL.randsvd(n, 1e4, 3, WL.rng_for(7, n))
    xh = x + 1e-9 * np.random.default_rng(1).standard_normal(n)
    r = OOPS.residual(A, xh, b, ur)
    s = OOPS.rnorm_inf(r)
    want = OOPS.scale_residual(r, s, u)
    rhat, sg = M.residual(h, dev(A, M), tdev(xh), tdev(b), ur, u)
    rg = rhat.cpu().numpy()
    if ur == "dd":
        assert abs(sg - s) <= 1e-15 * s
        mism = np.mean(rg != want)
        assert mism <= 0.05
        assert np.abs(rg - want).max() <= 4 * F.u(u)
    else:
        # float64 accumulation order differs: |r| agrees to n u_64 |A||x|
        bound = 4 * n * F.u("fp64") * (np.abs(A) @ np.abs(xh) + np.abs(b)).max()
        assert abs(sg - s) <= bound
        assert np.abs(rg * sg - want * s).max() <= bound + 2 * F.u(u) * s


def test_backward_error_vs_oracle(M, h):
    from oracle import metrics as OM
    n = 300
    A, x, b = WL.randsvd(n, 1e3, 2, WL.rng_for(8, 0))
    xh = x * (1 + 1e-12 * np.random.default_rng(2).standard_normal(n))
    nbe, cbe = M.backward_error(h, dev(A, M), tdev(xh), tdev(b))
    assert nbe == pytest.approx(OM.nbe(A, xh, b), rel=1e-10)
    assert cbe == pytest.approx(OM.cbe(A, xh, b), rel=1e-10)


# ------------------------------------------------------------------ GMRES
@pytest.mark.parametrize("u,p,restart", [("fp32", "fp32", 0), ("fp32", "fp64", 0), ("fp32", "fp32", 7),
                                         ("fp64", "fp64", 0), ("fp64", "dd", 0)])
def test_gmres_vs_oracle(M, h, u, p, restart):
    n = 160
    A, x, b = WL.randsvd(n, 1e5, 3, WL.rng_for(12, 0))
    Af = F.round_to(A, "fp16")
    W, piv, _ = OLU.getrf(Af, "fp16", 16)
    r = b - A @ (x + 1e-3 * np.random.default_rng(3).standard_normal(n))
    rhat = F.round_to(r / np.abs(r).max(), u)
    tau = 1e-6 if u == "fp32" else 1e-10
    dw, kw = OGM.gmres(A, W, piv, None, rhat, u, p, tau, 40, restart)
    Wd = to_dev_fmt(W, "fp16", M)
    ip = torch.from_numpy(piv.astype(np.int32)).to(DEV)
    dg, kg = M.gmres(h, dev(A, M), "fp16", Wd, ip, tdev(rhat), u, p, tau, 40, restart)
    dg = dg.cpu().numpy()
    assert abs(kg - kw) <= 1, (kg, kw)
    tol = 1e-3 if u == "fp32" else 1e-6
    assert np.abs(dg - dw).max() <= tol * np.abs(dw).max()


@pytest.mark.parametrize("comp", ["fp32", "fp64"])
@pytest.mark.parametrize("n,scaled", [(64, False), (150, True), (300, False)])
def test_getrs_explicit_inverse_mode(M, h, comp, n, scaled):
    # mode 1 applies M^{-1} through float64 inverses of L and U rounded to comp: the
    # same operator as substitution, differing by rounding amplified at most by the
    # condition numbers of the triangular factors.
    A, W, piv, scal = oracle_factors(n, "fp16", 16, 40 + n, scaled)
    t = np.random.default_rng(7).standard_normal(n)
    want = OSV.lu_solve(W, piv, t, "fp64", scal)
    Wd = to_dev_fmt(W, "fp16", M)
    ip = torch.from_numpy(piv.astype(np.int32)).to(DEV)
    R = S = None
    mu = 1.0
    if scal is not None:
        R, S, mu = tdev(scal[0]), tdev(scal[1]), scal[2]
    got = M.getrs(h, Wd, "fp16", ip, tdev(t), comp, R, S, mu, mode=1).cpu().numpy()
    L, U = OLU.unpack(W)
    kap = np.linalg.cond(L, np.inf) * np.linalg.cond(U, np.inf)
    rel = np.abs(got - want).max() / np.abs(want).max()
    assert rel <= 8 * n * kap * F.u(comp), (rel, kap)

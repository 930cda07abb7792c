"""The oracle's C loops (oracle/native) against its Python loops: the same blocked LU
(Alg. 4, first line) bit for bit, over factor formats, panel widths, ragged last
panels, ties, zero pivot columns and NaN entries.  The Python loops are pinned
against exact rational arithmetic in test_oracle_lu_rational.py."""
import numpy as np
import pytest

from oracle import fmt as F
from oracle import lu as LU
from oracle import native as NAT

pytestmark = pytest.mark.skipif(not NAT.available(), reason="oracle/native not built")


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32", "fp64"])
@pytest.mark.parametrize("n,nb", [(1, 8), (7, 2), (64, 16), (129, 32), (200, 8), (301, 64)])
def test_native_lu_equals_python(fmt, n, nb):
    rng = np.random.default_rng(1000 * n + nb)
    A = F.round_to(rng.standard_normal((n, n)) * np.exp2(rng.integers(-4, 5, (n, 1))), fmt)
    Wp, pp, ip = LU.getrf(A, fmt, nb, native=False)
    Wn, pn, inn = LU.getrf(A, fmt, nb, native=True)
    assert ip == inn
    np.testing.assert_array_equal(pp, pn)
    np.testing.assert_array_equal(Wp, Wn)


@pytest.mark.parametrize("fmt", ["fp16", "fp32", "fp64"])
def test_native_lu_special_cases(fmt):
    # ties (first index wins), a zero column (info, no scaling), NaN never chosen
    n = 40
    rng = np.random.default_rng(5)
    A = F.round_to(rng.integers(-3, 4, (n, n)).astype(float), fmt)
    A[:, 7] = 0.0
    A[3, 11] = np.nan
    Wp, pp, ip = LU.getrf(A, fmt, 16, native=False)
    Wn, pn, inn = LU.getrf(A, fmt, 16, native=True)
    assert ip == inn == 8
    np.testing.assert_array_equal(pp, pn)
    np.testing.assert_array_equal(Wp, Wn)     # NaN positions included (assert_array_equal treats NaN == NaN)

"""The C ABI library loads and exports every entry point declared in include/msir.h
(no device calls: this runs without a GPU)."""
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msir.h")
LIB = os.path.join(ROOT, "paper_2107_06200_amd", "libmsir.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"MSIR_API\s+[\w\s\*]*?\b(msir_\w+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for must in ("msir_solve", "msir_solve_multi", "msir_solve_batched", "msir_getrf", "msir_getrs",
                 "msir_residual", "msir_gmres", "msir_convert", "msir_create", "msir_destroy"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmsir.so not built")
def test_library_exports_every_declared_symbol():
    import ctypes
    L = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(L, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmsir.so not built")
def test_binding_signatures_cover_the_header():
    from paper_2107_06200_amd import msir as M
    M.lib()
    assert sorted(M.SYMBOLS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmsir.so not built")
def test_host_only_calls():
    # calls that touch no device: defaults, the panel-width rule, status strings
    from paper_2107_06200_amd import msir as M
    P = M.params()
    assert (P.uf, P.u, P.ur, P.ux, P.i_max, P.rho_thresh, P.restart) == (0, 2, 3, 3, 10, 0.5, 0)
    assert M.nb_auto(100, "fp16") == 64 and M.nb_auto(4096, "fp16") == 16 and M.nb_auto(8192, "fp16") == 8
    assert M.nb_auto(4096, "fp64") == 8
    assert M.lib().msir_status_string(0) == b"converged"
    assert M.workspace_bytes(1000) > 8 * 1000 * 1000


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmsir.so not built")
def test_panel_width_rule_agrees_with_oracle():
    # the oracle and the library state the same default panel-width rule independently
    from paper_2107_06200_amd import msir as M
    from oracle import lu as OLU
    for n in (1, 64, 100, 1024, 1025, 2048, 3000, 4096, 5000, 8192, 8193, 12000, 16384):
        for fmt in ("fp16", "bf16", "fp32", "fp64"):
            assert M.nb_auto(n, fmt) == OLU.nb_auto(n, fmt), (n, fmt)


def test_sparse_workload_is_valid_csr():
    # the synthetic sparse inputs: valid CSR (row pointers, sorted distinct columns in
    # range, diagonal present) that equals the dense matrix the oracle uses
    from paper_2107_06200_amd import workloads as WL
    rp, ci, v, A, x, b = WL.sparse_system(200, 6, 10.0, WL.rng_for(51, 200))
    n = 200
    assert rp[0] == 0 and rp[-1] == len(ci) == len(v) and np.all(np.diff(rp) >= 0)
    for i in range(n):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0) and cols.min() >= 0 and cols.max() < n and i in cols
    D = np.zeros((n, n))
    for i in range(n):
        D[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    assert np.array_equal(D, A)
    assert np.allclose(A @ x, b)

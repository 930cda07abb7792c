"""The allocation-free residual entry point against msir_residual (the entry point it
is a variant of): the same kernels on the same inputs, so rhat and s must be equal bit
for bit.  Two calls in a row, the second with a smaller order (the shared scratch array
keeps the first call's contents), in both residual precisions, up to the largest
order the array serves; an order above it is refused before any device work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def system(n, seed):
    g = torch.Generator(device=DEV).manual_seed(seed)
    A = torch.randn((n, n), generator=g, device=DEV, dtype=torch.float64)
    x = torch.randn(n, generator=g, device=DEV, dtype=torch.float64)
    b = torch.randn(n, generator=g, device=DEV, dtype=torch.float64)
    return A.t().contiguous().t(), x, b


@pytest.mark.parametrize("ur,u", [("fp64", "fp32"), ("dd", "fp64")])
@pytest.mark.parametrize("sizes", [(8192, 1000), (4096, 37), (513, 512)])
def test_noalloc_residual_equals_residual(M, h, ur, u, sizes):
    for k, n in enumerate(sizes):
        A, x, b = system(n, 100 * k + n)
        print("noalloc residual n=%d ur=%s u=%s" % (n, ur, u), flush=True)
        r0, s0 = M.residual(h, A, x, b, ur, u)
        r1, s1 = M.residual_noalloc(h, A, x, b, ur, u)
        torch.cuda.synchronize()
        assert s1 == s0 and s1 > 0
        assert torch.equal(r1, r0)


def test_noalloc_residual_first_call_on_a_fresh_handle(M):
    # the handle's own workspace is never grown: the call works as the first one
    hh = M.Handle(0)
    try:
        A, x, b = system(300, 7)
        r1, s1 = M.residual_noalloc(hh, A, x, b, "fp64", "fp64")
        r0, s0 = M.residual(hh, A, x, b, "fp64", "fp64")
        assert s1 == s0 and torch.equal(r1, r0)
    finally:
        hh.close()


def test_noalloc_residual_refuses_orders_above_its_array(M, h):
    n = 8193
    A = torch.zeros((1, 1), device=DEV, dtype=torch.float64)
    # refused by the host-side size check before any device work (the pointers are
    # never dereferenced)
    rc = M.lib().msir_residual_noalloc(h.h, n, M._ptr(A), n, M._ptr(A), M._ptr(A), 3, 3, M._ptr(A), None)
    assert rc == -102

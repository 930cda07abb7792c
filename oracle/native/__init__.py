"""Plain C forms of oracle steps whose Python loops are too slow at the workloads'
full orders (test infrastructure only; built by ``python -m oracle.native.build``).

``getrf`` is the blocked LU of ``oracle.lu`` as plain loops (dm_lu.c); the tests pin
it bit for bit against the Python form.  Nothing here imports or links the product.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_FMT = {"fp16": 0, "bf16": 1, "fp32": 2, "fp64": 3}


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libdm_lu.so")
        if not os.path.exists(path):
            return None
        L = ctypes.CDLL(path)
        L.dm_getrf.restype = ctypes.c_int
        L.dm_getrf.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        _LIB = L
    return _LIB


def available():
    return _lib() is not None


def getrf(A, fmt_f, nb):
    """(W, piv, info) of the blocked LU (see oracle.lu.getrf), computed by dm_lu.c."""
    L = _lib()
    if L is None:
        raise RuntimeError("oracle/native/libdm_lu.so is not built (python -m oracle.native.build)")
    W = np.array(A, dtype=np.float64, order="F", copy=True)
    n = W.shape[0]
    piv = np.arange(n, dtype=np.int64)
    info = L.dm_getrf(n, W.ctypes.data, _FMT[fmt_f], int(nb), piv.ctypes.data)
    return W, piv, int(info)

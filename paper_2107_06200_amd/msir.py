"""ctypes binding of libmsir (include/msir.h): argument marshalling only.

Every numerical step runs in the HIP library; this module converts torch
tensors to device pointers, fills the C structs and checks return codes.  It
raises if the library is missing: there is no fallback path.

Matrices are column-major.  A square matrix argument may be any (n, n) torch
tensor on the handle's device: a column-major one (strides (1, n)) is used in
place, anything else is copied to column-major first.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libmsir.so")
_LIB = None

PREC = {"fp16": 0, "bf16": 1, "fp32": 2, "fp64": 3, "dd": 4}
PREC_NAME = {v: k for k, v in PREC.items()}
CONV = {"estimate": 0, "backward": 1, "true": 2, "componentwise": 3}
SCALE = {"never": 0, "auto": 1, "always": 2, "cols": 3}
TORCH_DTYPE = {0: torch.float16, 1: torch.bfloat16, 2: torch.float32, 3: torch.float64}
STATUS = {0: "converged", 1: "not converged", 2: "singular"}

EV_NAN_D, EV_RESET_X0, EV_SWITCH, EV_ESCALATE, EV_SCALED, EV_NAN_X0, EV_CONVERGED = 1, 2, 4, 8, 16, 32, 64


class Params(ctypes.Structure):
    _fields_ = [("uf", ctypes.c_int), ("u", ctypes.c_int), ("ur", ctypes.c_int), ("ux", ctypes.c_int),
                ("i_max", ctypes.c_int), ("tau", ctypes.c_double), ("rho_thresh", ctypes.c_double),
                ("k_max", ctypes.c_double), ("restart", ctypes.c_int), ("conv", ctypes.c_int),
                ("tol_nbe", ctypes.c_double), ("scaling", ctypes.c_int), ("nb", ctypes.c_int),
                ("max_steps", ctypes.c_int), ("lu_update", ctypes.c_int), ("gmres_op", ctypes.c_int)]


class Step(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("uf", ctypes.c_int), ("u", ctypes.c_int), ("ur", ctypes.c_int),
                ("stage", ctypes.c_int), ("iter", ctypes.c_int), ("k_gmres", ctypes.c_int), ("counted", ctypes.c_int),
                ("z", ctypes.c_double), ("v", ctypes.c_double), ("rho_max", ctypes.c_double), ("phi", ctypes.c_double),
                ("rnorm", ctypes.c_double), ("nbe", ctypes.c_double), ("events", ctypes.c_uint)]


class Result(ctypes.Structure):
    _fields_ = [("cged", ctypes.c_int), ("status", ctypes.c_int), ("steps", ctypes.c_int), ("n_lu", ctypes.c_int),
                ("gmres_iters", ctypes.c_int), ("final_uf", ctypes.c_int), ("final_u", ctypes.c_int),
                ("final_ur", ctypes.c_int), ("nbe", ctypes.c_double), ("ferr", ctypes.c_double),
                ("cbe", ctypes.c_double), ("t_factor_ms", ctypes.c_double), ("t_refine_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int), ("n", ctypes.c_int), ("nrhs", ctypes.c_int), ("dA", ctypes.c_void_p),
                ("lda", ctypes.c_int), ("dB", ctypes.c_void_p), ("ldb", ctypes.c_int), ("dX", ctypes.c_void_p),
                ("ldx", ctypes.c_int)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int), ("status", ctypes.c_int), ("nrhs", ctypes.c_int), ("slot", ctypes.c_int),
                ("n_lu", ctypes.c_int), ("gmres_iters", ctypes.c_int), ("nbe_max", ctypes.c_double),
                ("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double), ("t_end_ms", ctypes.c_double)]


SYMBOLS = ["msir_create", "msir_destroy", "msir_params_default", "msir_nb_auto", "msir_workspace_bytes",
           "msir_status_string", "msir_solve", "msir_solve_csr", "msir_gmres_ir5", "msir_lstsq", "msir_solve_multi", "msir_solve_batched", "msir_convert",
           "msir_scaling", "msir_getrf", "msir_getrs", "msir_round", "msir_residual", "msir_residual_noalloc", "msir_gmres", "msir_backward_error",
           "msir_timing", "msir_timing_get", "msir_server_create", "msir_server_submit", "msir_server_poll",
           "msir_server_destroy"]

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIG = {
    "msir_create": (_I, [ctypes.POINTER(_P), _I, ctypes.c_size_t, _P]),
    "msir_server_create": (_I, [ctypes.POINTER(_P), _I, _I, ctypes.c_size_t, ctypes.POINTER(Params)]),
    "msir_server_submit": (_I, [_P, ctypes.POINTER(Request)]),
    "msir_server_poll": (_I, [_P, ctypes.POINTER(Completion), _I, ctypes.POINTER(_I), _I]),
    "msir_server_destroy": (_I, [_P]),
    "msir_destroy": (_I, [_P]),
    "msir_params_default": (None, [ctypes.POINTER(Params)]),
    "msir_nb_auto": (_I, [_I, _I]),
    "msir_workspace_bytes": (ctypes.c_size_t, [_I, ctypes.POINTER(Params)]),
    "msir_status_string": (ctypes.c_char_p, [_I]),
    "msir_solve": (_I, [_P, _I, _P, _I, _P, _P, _P, ctypes.POINTER(Params), ctypes.POINTER(Result),
                        ctypes.POINTER(Step), _I, ctypes.POINTER(_I)]),
    "msir_solve_csr": (_I, [_P, _I, _I, _P, _P, _P, _P, _P, _P, ctypes.POINTER(Params), ctypes.POINTER(Result),
                            ctypes.POINTER(Step), _I, ctypes.POINTER(_I)]),
    "msir_gmres_ir5": (_I, [_P, _I, _P, _I, _P, _P, _P, ctypes.POINTER(Params), _I, _I, ctypes.POINTER(Result),
                            ctypes.POINTER(Step), _I, ctypes.POINTER(_I)]),
    "msir_lstsq": (_I, [_P, _I, _I, _P, _I, _P, _D, _P, _P, ctypes.POINTER(_D), ctypes.POINTER(Params),
                        ctypes.POINTER(Result), ctypes.POINTER(Step), _I, ctypes.POINTER(_I)]),
    "msir_solve_multi": (_I, [_P, _I, _I, _P, _I, _P, _I, _P, _I, _P, _I, ctypes.POINTER(Params),
                              ctypes.POINTER(Result), ctypes.POINTER(Step), _I, ctypes.POINTER(_I)]),
    "msir_solve_batched": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_P), ctypes.POINTER(_I),
                                ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(Params),
                                ctypes.POINTER(Result), ctypes.POINTER(Step), _I, ctypes.POINTER(_I)]),
    "msir_convert": (_I, [_P, _I, _P, _I, _I, _P, _P, _D, _P, _I]),
    "msir_scaling": (_I, [_P, _I, _P, _I, _I, _I, _P, _P, _P]),
    "msir_getrf": (_I, [_P, _I, _I, _P, _I, _I, _I, _P, ctypes.POINTER(_I)]),
    "msir_getrs": (_I, [_P, _I, _I, _P, _I, _P, _P, _P, _D, _I, _I, _P, _P]),
    "msir_round": (_I, [_P, _I, _I, _P, _P]),
    "msir_residual": (_I, [_P, _I, _P, _I, _P, _P, _I, _I, _P, ctypes.POINTER(_D)]),
    "msir_residual_noalloc": (_I, [_P, _I, _P, _I, _P, _P, _I, _I, _P, ctypes.POINTER(_D)]),
    "msir_gmres": (_I, [_P, _I, _P, _I, _I, _P, _I, _P, _P, _P, _D, _P, _I, _I, _D, _D, _I, _P,
                        ctypes.POINTER(_I)]),
    "msir_backward_error": (_I, [_P, _I, _P, _I, _P, _P, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "msir_timing": (_I, [_P, _I]),
    "msir_timing_get": (_I, [_P, _I, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_D)]),
}

TIMERS = ["panel", "swap", "gemm", "trsv", "matvec32", "resid", "arnoldi", "trgemv32", "fold", "matvec64",
          "trgemv64"]


def lib(path=None):
    """Load libmsir.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    p = path or LIBPATH
    if not os.path.exists(p):
        raise RuntimeError("libmsir.so not found at %s: build it with __graft_entry__.build()" % p)
    L = ctypes.CDLL(p)
    for name, (res, args) in _SIG.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


class MsirError(RuntimeError):
    pass


def _check(rc, what):
    if rc < 0:
        raise MsirError("%s failed: %d (%s)" % (what, rc, lib().msir_status_string(rc).decode()))
    return rc


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def colmajor(A):
    """Column-major (Fortran-order) version of a 2-D tensor (no copy if it already is;
    a single column with unit row stride is column-major whatever its column stride)."""
    if A.dim() == 2 and A.stride(0) == 1 and (A.shape[1] == 1 or A.stride(1) >= max(1, A.shape[0])):
        return A
    out = torch.empty_strided(tuple(A.shape), (1, max(1, A.shape[0])), dtype=A.dtype, device=A.device)
    out.copy_(A)
    return out


def _ld(A):
    """Leading dimension of a column-major tensor (its rows for a single column)."""
    return A.stride(1) if A.shape[1] > 1 else max(1, A.shape[0])


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)


def params(**kw):
    """msir_params from keyword overrides of the library defaults (names of include/msir.h;
    precisions and modes may be given by name)."""
    P = Params()
    lib().msir_params_default(ctypes.byref(P))
    for k, v in kw.items():
        if v is None:
            continue
        if k in ("uf", "u", "ur", "ux"):
            v = _prec(v)
        elif k == "conv" and isinstance(v, str):
            v = CONV[v]
        elif k == "scaling" and isinstance(v, str):
            v = SCALE[v]
        elif k == "lu_update" and isinstance(v, str):
            v = {"mfma": 0, "fma": 1}[v]
        elif k == "gmres_op" and isinstance(v, str):
            v = {"inverse": 0, "subst": 1}[v]
        setattr(P, k, v)
    return P


class Handle:
    """An msir_handle bound to one device and the current torch stream."""

    def __init__(self, device=0, budget=0, stream=None):
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = ctypes.c_void_p()
        _check(L.msir_create(ctypes.byref(h), device, budget, ctypes.c_void_p(stream.cuda_stream)), "msir_create")
        self.h = h

    def close(self):
        if self.h:
            lib().msir_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nb_auto(n, fmt):
    return lib().msir_nb_auto(n, _prec(fmt))


def workspace_bytes(n, P=None):
    return lib().msir_workspace_bytes(n, ctypes.byref(P) if P is not None else None)


def solve(h, A, b, x_true=None, P=None, hist_cap=4096, x=None):
    """Alg. 4 on A x = b.  Returns (x, Result, [Step...], status)."""
    A = colmajor(A)
    n = A.shape[0]
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=A.device)
    res = Result()
    H = (Step * hist_cap)()
    hl = ctypes.c_int(0)
    rc = lib().msir_solve(h.h, n, _ptr(A), _ld(A), _ptr(b), _ptr(x), _ptr(x_true),
                          ctypes.byref(P) if P is not None else None, ctypes.byref(res), H, hist_cap,
                          ctypes.byref(hl))
    _check(rc, "msir_solve")
    return x, res, [H[i] for i in range(min(hl.value, hist_cap))], rc


def solve_csr(h, rowptr, colind, vals, b, x_true=None, P=None, hist_cap=4096, x=None):
    """Alg. 4 with a sparse A in CSR form (int32 rowptr/colind, float64 vals, device
    tensors).  Returns (x, Result, [Step...], status)."""
    n = rowptr.shape[0] - 1
    nnz = colind.shape[0]
    for t, dt in ((rowptr, torch.int32), (colind, torch.int32), (vals, torch.float64)):
        if t.dtype != dt or not t.is_contiguous():
            raise ValueError("solve_csr: rowptr/colind int32, vals float64, contiguous")
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=b.device)
    res = Result()
    H = (Step * hist_cap)()
    hl = ctypes.c_int(0)
    rc = lib().msir_solve_csr(h.h, n, nnz, _ptr(rowptr), _ptr(colind), _ptr(vals), _ptr(b), _ptr(x), _ptr(x_true),
                              ctypes.byref(P) if P is not None else None, ctypes.byref(res), H, hist_cap,
                              ctypes.byref(hl))
    _check(rc, "msir_solve_csr")
    return x, res, [H[i] for i in range(min(hl.value, hist_cap))], rc


def gmres_ir5(h, A, b, ug, up, x_true=None, P=None, hist_cap=4096, x=None):
    """GMRES-IR5 with GMRES precision ug and operator precision up (names or
    msir_prec values).  Returns (x, Result, [Step...], status)."""
    A = colmajor(A)
    n = A.shape[0]
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=A.device)
    res = Result()
    H = (Step * hist_cap)()
    hl = ctypes.c_int(0)
    rc = lib().msir_gmres_ir5(h.h, n, _ptr(A), _ld(A), _ptr(b), _ptr(x), _ptr(x_true),
                              ctypes.byref(P) if P is not None else None, _prec(ug), _prec(up), ctypes.byref(res),
                              H, hist_cap, ctypes.byref(hl))
    _check(rc, "msir_gmres_ir5")
    return x, res, [H[i] for i in range(min(hl.value, hist_cap))], rc


def lstsq(h, A, b, alpha=0.0, P=None, hist_cap=4096, x=None, r=None):
    """min ||b - A x||_2 by Alg. 4 on the augmented system (A m x n, m >= n).
    Returns (x, r, alpha used, Result, [Step...], status)."""
    A = colmajor(A)
    m, n = A.shape
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=A.device)
    if r is None:
        r = torch.empty(m, dtype=torch.float64, device=A.device)
    res = Result()
    H = (Step * hist_cap)()
    hl = ctypes.c_int(0)
    au = ctypes.c_double(0.0)
    rc = lib().msir_lstsq(h.h, m, n, _ptr(A), _ld(A), _ptr(b), float(alpha), _ptr(x), _ptr(r), ctypes.byref(au),
                          ctypes.byref(P) if P is not None else None, ctypes.byref(res), H, hist_cap,
                          ctypes.byref(hl))
    _check(rc, "msir_lstsq")
    return x, r, au.value, res, [H[i] for i in range(min(hl.value, hist_cap))], rc


def solve_multi(h, A, B, X_true=None, P=None, hist_cap=512, X=None):
    """Alg. 4 for the columns of B over one factor cache.  Returns
    (X, [Result per column], [[Step...] per column], worst status)."""
    A = colmajor(A)
    B = colmajor(B)
    n, nrhs = B.shape
    if X is None:
        X = colmajor(torch.empty(n, nrhs, dtype=torch.float64, device=A.device))
    Xt = colmajor(X_true) if X_true is not None else None
    outs = (Result * nrhs)()
    H = (Step * (hist_cap * nrhs))()
    hl = (ctypes.c_int * nrhs)()
    rc = lib().msir_solve_multi(h.h, n, nrhs, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(X), _ld(X), _ptr(Xt),
                                _ld(Xt) if Xt is not None else n, ctypes.byref(P) if P is not None else None,
                                outs, H, hist_cap, hl)
    _check(rc, "msir_solve_multi")
    hists = [[H[j * hist_cap + i] for i in range(min(hl[j], hist_cap))] for j in range(nrhs)]
    return X, [outs[i] for i in range(nrhs)], hists, rc


def solve_batched(h, As, bs, x_true=None, P=None, hist_cap=256, xs=None):
    """Alg. 4 for independent systems (As[i], bs[i]).  Returns
    (xs, [Result per system], [[Step...] per system], worst status)."""
    count = len(As)
    As = [colmajor(A) for A in As]
    if xs is None:
        xs = [torch.empty(A.shape[0], dtype=torch.float64, device=A.device) for A in As]
    ns = (ctypes.c_int * count)(*[A.shape[0] for A in As])
    ld = (ctypes.c_int * count)(*[_ld(A) for A in As])
    pA = (ctypes.c_void_p * count)(*[A.data_ptr() for A in As])
    pb = (ctypes.c_void_p * count)(*[b.data_ptr() for b in bs])
    px = (ctypes.c_void_p * count)(*[x.data_ptr() for x in xs])
    pt = (ctypes.c_void_p * count)(*[t.data_ptr() for t in x_true]) if x_true is not None else None
    outs = (Result * count)()
    H = (Step * (hist_cap * count))()
    hl = (ctypes.c_int * count)()
    rc = lib().msir_solve_batched(h.h, count, ns, pA, ld, pb, px, pt, ctypes.byref(P) if P is not None else None,
                                  outs, H, hist_cap, hl)
    _check(rc, "msir_solve_batched")
    hists = [[H[i * hist_cap + k] for k in range(min(hl[i], hist_cap))] for i in range(count)]
    return xs, [outs[i] for i in range(count)], hists, rc


def convert(h, A, fmt, R=None, S=None, mu=1.0):
    """fl_fmt(mu R A S) as a column-major tensor of the format's torch dtype (bit patterns)."""
    A = colmajor(A)
    n = A.shape[0]
    f = _prec(fmt)
    W = colmajor(torch.empty(n, n, dtype=TORCH_DTYPE[f], device=A.device))
    if R is not None:
        import numpy as np
        R = np.ascontiguousarray(R, dtype=np.float64)
        S = np.ascontiguousarray(S, dtype=np.float64)
        rp, sp = R.ctypes.data_as(ctypes.c_void_p), S.ctypes.data_as(ctypes.c_void_p)
    else:
        rp = sp = None
    _check(lib().msir_convert(h.h, n, _ptr(A), _ld(A), f, rp, sp, float(mu), _ptr(W), _ld(W)), "msir_convert")
    return W


def scaling(h, A, fmt, rows=True):
    import numpy as np
    A = colmajor(A)
    n = A.shape[0]
    R = np.empty(n)
    S = np.empty(n)
    mu = ctypes.c_double(0)
    _check(lib().msir_scaling(h.h, n, _ptr(A), _ld(A), _prec(fmt), 1 if rows else 0,
                              R.ctypes.data_as(ctypes.c_void_p), S.ctypes.data_as(ctypes.c_void_p),
                              ctypes.byref(mu)), "msir_scaling")
    return R, S, mu.value


LU_UPDATE = {"mfma": 0, "fma": 1}


def getrf(h, W, fmt, nb=0, update="mfma"):
    """In-place LU of W (column-major, format fmt).  Returns (ipiv int32 tensor, info)."""
    assert W.stride(0) == 1
    n = W.shape[0]
    ipiv = torch.empty(n, dtype=torch.int32, device=W.device)
    info = ctypes.c_int(0)
    _check(lib().msir_getrf(h.h, n, _prec(fmt), _ptr(W), _ld(W), nb, LU_UPDATE[update], _ptr(ipiv),
                            ctypes.byref(info)), "msir_getrf")
    return ipiv, info.value


def getrs(h, W, fmt, ipiv, t, comp, R=None, S=None, mu=1.0, mode=0):
    """mu S U^{-1} L^{-1} P R t with components rounded to comp (t: float64, 2n for 'dd')."""
    n = W.shape[0]
    c = _prec(comp)
    y = torch.empty(2 * n if c == 4 else n, dtype=torch.float64, device=W.device)
    _check(lib().msir_getrs(h.h, n, _prec(fmt), _ptr(W), _ld(W), _ptr(ipiv), _ptr(R), _ptr(S), float(mu), c, mode,
                            _ptr(t), _ptr(y)), "msir_getrs")
    return y


def round_values(h, x, fmt):
    """fl_fmt(x) for a float64 device vector (new tensor)."""
    import torch
    assert x.dtype == torch.float64 and x.is_contiguous()
    y = torch.empty_like(x)
    _check(lib().msir_round(h.h, x.numel(), _prec(fmt), _ptr(x), _ptr(y)), "msir_round")
    return y


def residual(h, A, x, b, ur, u):
    A = colmajor(A)
    n = A.shape[0]
    rhat = torch.empty(n, dtype=torch.float64, device=A.device)
    s = ctypes.c_double(0)
    _check(lib().msir_residual(h.h, n, _ptr(A), _ld(A), _ptr(x), _ptr(b), _prec(ur), _prec(u), _ptr(rhat),
                               ctypes.byref(s)), "msir_residual")
    return rhat, s.value


def residual_noalloc(h, A, x, b, ur, u, rhat=None):
    """msir_residual_noalloc: as residual(), with the library's fixed scratch array."""
    A = colmajor(A)
    n = A.shape[0]
    if rhat is None:
        rhat = torch.empty(n, dtype=torch.float64, device=A.device)
    s = ctypes.c_double(0)
    _check(lib().msir_residual_noalloc(h.h, n, _ptr(A), _ld(A), _ptr(x), _ptr(b), _prec(ur), _prec(u), _ptr(rhat),
                                       ctypes.byref(s)), "msir_residual_noalloc")
    return rhat, s.value


def gmres(h, A, fmt, W, ipiv, rhat, u, p, tau, k_max, restart=0, R=None, S=None, mu=1.0):
    A = colmajor(A)
    n = A.shape[0]
    d = torch.empty(n, dtype=torch.float64, device=A.device)
    k = ctypes.c_int(0)
    _check(lib().msir_gmres(h.h, n, _ptr(A), _ld(A), _prec(fmt), _ptr(W), _ld(W), _ptr(ipiv), _ptr(R), _ptr(S),
                            float(mu), _ptr(rhat), _prec(u), _prec(p), float(tau), float(k_max), int(restart),
                            _ptr(d), ctypes.byref(k)), "msir_gmres")
    return d, k.value


def backward_error(h, A, x, b):
    A = colmajor(A)
    n = A.shape[0]
    nbe = ctypes.c_double(0)
    cbe = ctypes.c_double(0)
    _check(lib().msir_backward_error(h.h, n, _ptr(A), _ld(A), _ptr(x), _ptr(b), ctypes.byref(nbe),
                                     ctypes.byref(cbe)), "msir_backward_error")
    return nbe.value, cbe.value


def timing(h, enable=True):
    _check(lib().msir_timing(h.h, 1 if enable else 0), "msir_timing")


def timing_get(h):
    """{class name: (launches, total device ms)} since timing was enabled."""
    out = {}
    for i, name in enumerate(TIMERS):
        c = ctypes.c_longlong(0)
        t = ctypes.c_double(0)
        _check(lib().msir_timing_get(h.h, i, ctypes.byref(c), ctypes.byref(t)), "msir_timing_get")
        out[name] = (c.value, t.value)
    return out


class Server:
    """msir_server: requests (A, B) solved concurrently in `slots` service slots under a
    device-memory budget.  The caller keeps the tensors of a request alive until its
    completion has been returned by poll()."""

    def __init__(self, device=0, slots=4, budget=0, P=None):
        self.s = ctypes.c_void_p()
        _check(lib().msir_server_create(ctypes.byref(self.s), device, slots, budget,
                                        ctypes.byref(P) if P is not None else None), "msir_server_create")
        self.keep = {}

    def submit(self, rid, A, B, X):
        A, B, X = colmajor(A), colmajor(B), colmajor(X)
        r = Request(rid, A.shape[0], B.shape[1], A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), X.data_ptr(), _ld(X))
        self.keep[rid] = (A, B, X)
        _check(lib().msir_server_submit(self.s, ctypes.byref(r)), "msir_server_submit")

    def poll(self, cap=64, wait_ms=0):
        """(completions, outstanding)"""
        out = (Completion * cap)()
        cnt = ctypes.c_int(0)
        rem = lib().msir_server_poll(self.s, out, cap, ctypes.byref(cnt), wait_ms)
        _check(rem, "msir_server_poll")
        comps = [out[i] for i in range(cnt.value)]
        for c in comps:
            self.keep.pop(c.id, None)
        return comps, rem

    def close(self):
        if self.s:
            lib().msir_server_destroy(self.s)
            self.s = ctypes.c_void_p()


def render(steps):
    """The paper's notation for a history (e.g. '2, (5,10), (10); 2, (2,2,2)')."""
    levels = []
    cur = None
    for st in steps:
        if cur is None or st.level != cur[0]:
            cur = (st.level, [0, [], []])
            levels.append(cur)
        if st.stage == 0:
            if st.counted:
                cur[1][0] += 1
        elif st.counted:
            cur[1][st.stage].append(st.k_gmres)
    parts = []
    for _, d in levels:
        items = [str(d[0])] + ["(" + ",".join(str(k) for k in d[s]) + ")" for s in (1, 2) if d[s]]
        parts.append(", ".join(items))
    return "; ".join(parts)

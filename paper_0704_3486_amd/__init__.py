"""Python binding of libsgn: y = sgn(H_w(mu)) x on an MI355X (gfx950).

The functions below carry the names of the C ABI in include/sgn.h and only
marshal arguments: device vectors are torch tensors (complex128, on the GPU),
host arrays are numpy arrays.  Every computation runs in the HIP library;
importing this package fails loudly if libsgn.so has not been built.

    import torch, paper_0704_3486_amd as sg
    ctx = sg.sgn_create(links, (L, L, L, L), mu, m_w)     # links: numpy (V,4,3,3)
    sg.sgn_deflate_import(ctx, S, T)                       # optional deflation
    y = torch.empty_like(x); sg.sgn_apply(ctx, x, y, 1e-10, 500)
    sg.sgn_destroy(ctx)
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgn.so")

SGN_OK = 0
SGN_EINVAL = -1
SGN_ENOMEM = -2
SGN_EHIP = -3
SGN_ENOCONV = -4
SGN_ESINGULAR = -5
SGN_ESTATE = -6
SGN_EDEFL = -7
SGN_DEFL_NONE = 0
SGN_DEFL_SCHUR = 1
SGN_DEFL_LR = 2
SGN_SIGN_SCHULZ = 0
SGN_SIGN_ROBERTS = 1
SGN_ORTH_CGS2 = 0
SGN_ORTH_DELAYED = 1
SGN_PREC_FP64 = 0
SGN_PREC_MIXED = 1


class sgn_info(C.Structure):
    _fields_ = [
        ("k_used", C.c_int), ("converged", C.c_int), ("newton_iters", C.c_int), ("n_matvec", C.c_int),
        ("n_checkpoints", C.c_int), ("breakdown", C.c_int),
        ("err_est", C.c_double), ("beta", C.c_double), ("ms_arnoldi", C.c_double), ("ms_sign", C.c_double),
        ("ms_total", C.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class sgn_kstat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_longlong), ("ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double)]


class SgnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it first (python paper_0704_3486_amd/build.py); "
            "there is no fallback implementation")
    lib = C.CDLL(LIB_PATH)
    vp, i, d, cp = C.c_void_p, C.c_int, C.c_double, C.c_char_p
    sig = {
        "sgn_create": (vp, [vp, C.POINTER(C.c_int), d, d]),
        "sgn_create_error": (cp, []),
        "sgn_destroy": (None, [vp]),
        "sgn_set_stream": (i, [vp, vp]),
        "sgn_get_dims": (i, [vp, C.POINTER(C.c_int), C.POINTER(C.c_longlong)]),
        "sgn_deflate_import": (i, [vp, i, vp, vp]),
        "sgn_deflate_export": (i, [vp, vp, vp, vp]),
        "sgn_deflation_size": (i, [vp]),
        "sgn_apply": (i, [vp, vp, vp, d, i]),
        "sgn_apply_fixed": (i, [vp, vp, vp, i]),
        "sgn_apply_adjoint": (i, [vp, vp, vp, d, i]),
        "sgn_apply_adjoint_fixed": (i, [vp, vp, vp, i]),
        "sgn_overlap_apply_adjoint": (i, [vp, vp, vp, d, i]),
        "sgn_overlap_solve": (i, [vp, vp, vp, d, d, i, i, d, i, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
        "sgn_apply_batched": (i, [vp, i, vp, vp, d, i, C.POINTER(sgn_info)]),
        "sgn_overlap_apply": (i, [vp, vp, vp, d, i]),
        "sgn_overlap_apply_batched": (i, [vp, i, vp, vp, d, i, C.POINTER(sgn_info)]),
        "sgn_session_create": (vp, [vp, i, i]),
        "sgn_session_submit": (i, [vp, vp, vp, d, i, C.POINTER(C.c_int)]),
        "sgn_session_step": (i, [vp, i]),
        "sgn_session_poll": (i, [vp, i, C.POINTER(sgn_info)]),
        "sgn_session_active": (i, [vp]),
        "sgn_session_destroy": (None, [vp]),
        "sgn_apply_batched_fixed": (i, [vp, i, vp, vp, i, C.POINTER(sgn_info)]),
        "sgn_apply_adjoint_batched": (i, [vp, i, vp, vp, d, i, C.POINTER(sgn_info)]),
        "sgn_apply_adjoint_batched_fixed": (i, [vp, i, vp, vp, i, C.POINTER(sgn_info)]),
        "sgn_last_info": (i, [vp, C.POINTER(sgn_info)]),
        "sgn_footprint_bytes": (C.c_size_t, [vp, i, i]),
        "sgn_matvec": (i, [vp, vp, vp]),
        "sgn_matvec_noalloc": (i, [vp, vp, vp]),
        "sgn_zgemm": (i, [vp, i, i, i, vp, i, vp, i, vp, i]),
        "sgn_dense_sign": (i, [vp, i, vp, vp, C.POINTER(C.c_int)]),
        "sgn_set_profiling": (i, [vp, i]),
        "sgn_profile_read": (i, [vp, C.POINTER(sgn_kstat), i]),
        "sgn_profile_reset": (i, [vp]),
        "sgn_deflate": (i, [vp, i]),
        "sgn_deflate_lr": (i, [vp, i]),
        "sgn_set_deflation_krylov": (i, [vp, i]),
        "sgn_set_deflation_filter": (i, [vp, i, d]),
        "sgn_deflate_filter_stats": (i, [vp, C.POINTER(C.c_int), C.POINTER(d), C.POINTER(d)]),
        "sgn_deflate_lr_import": (i, [vp, i, vp, vp, vp]),
        "sgn_deflate_lr_export": (i, [vp, vp, vp, vp]),
        "sgn_deflation_mode": (i, [vp]),
        "sgn_set_orthogonalization": (i, [vp, i]),
        "sgn_set_block_steps": (i, [vp, i]),
        "sgn_get_block_steps": (i, [vp, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
        "sgn_set_tuning": (i, [vp, i, i, i]),
        "sgn_set_step_graphs": (i, [vp, i]),
        "sgn_set_stencil_blocks": (i, [vp, i, i, i]),
        "sgn_get_tuning": (i, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "sgn_set_precision": (i, [vp, i]),
        "sgn_get_precision": (i, [vp]),
        "sgn_set_schedule": (i, [vp, i, d]),
        "sgn_set_sign_method": (i, [vp, i]),
        "sgn_deflate_stats": (i, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(d)]),
        "sgn_host_eig": (i, [i, vp, vp, vp]),
        "sgn_debug_hessenberg": (i, [vp, i, vp, vp, vp]),
        "sgn_strerror": (cp, [i]),
        "sgn_last_error": (cp, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
lib = _lib


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------
def _dptr(t, n=None, name="tensor"):
    """Device pointer of a contiguous complex128 CUDA/HIP tensor."""
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if t.dtype != torch.complex128 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous complex128")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} entries, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _hptr(a, n=None, name="array"):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if n is not None and a.size != n:
        raise ValueError(f"{name} must have {n} entries, has {a.size}")
    return a, a.ctypes.data_as(C.c_void_p)


def _check(ctx, st, soft=()):
    if st == SGN_OK or st in soft:
        return st
    msg = _lib.sgn_last_error(ctx).decode() if ctx else ""
    raise SgnError(st, f"{_lib.sgn_strerror(st).decode()}: {msg}")


# ---------------------------------------------------------------------------
# ABI functions (same names as include/sgn.h)
# ---------------------------------------------------------------------------
def sgn_create(gauge, dims, mu, m_w, stream=None):
    """Create a context; gauge is the host link array U[n][nu][3][3] (complex128).

    The context runs on torch's current stream unless another stream is given.
    """
    import torch

    dims = [int(d) for d in dims]
    V = dims[0] * dims[1] * dims[2] * dims[3]
    g, gp = _hptr(gauge, 36 * V, "gauge")
    cd = (C.c_int * 4)(*dims)
    ctx = _lib.sgn_create(gp, cd, float(mu), float(m_w))
    if not ctx:
        raise SgnError(SGN_EINVAL, _lib.sgn_create_error().decode())
    ctx = C.c_void_p(ctx)
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(ctx, _lib.sgn_set_stream(ctx, C.c_void_p(s)))
    return ctx


def sgn_destroy(ctx):
    _lib.sgn_destroy(ctx)


def sgn_set_stream(ctx, stream):
    return _check(ctx, _lib.sgn_set_stream(ctx, C.c_void_p(stream)))


def sgn_get_dims(ctx):
    d = (C.c_int * 4)()
    n = C.c_longlong()
    _check(ctx, _lib.sgn_get_dims(ctx, d, C.byref(n)))
    return tuple(d), int(n.value)


def sgn_deflate(ctx, m):
    """Compute and install the m critical Schur vectors on the device."""
    return _check(ctx, _lib.sgn_deflate(ctx, int(m)))


def sgn_deflate_stats(ctx):
    r, mv, res = C.c_int(), C.c_int(), C.c_double()
    _check(ctx, _lib.sgn_deflate_stats(ctx, C.byref(r), C.byref(mv), C.byref(res)))
    out = {"restarts": r.value, "matvecs": mv.value, "residual": res.value}
    out.update(sgn_deflate_filter_stats(ctx))
    return out


def sgn_deflate_filter_stats(ctx):
    deg, a, b = C.c_int(), C.c_double(), C.c_double()
    _check(ctx, _lib.sgn_deflate_filter_stats(ctx, C.byref(deg), C.byref(a), C.byref(b)))
    return {"filter_degree": deg.value, "filter_interval": [a.value, b.value]}


def sgn_deflate_import(ctx, S, T):
    """Install (S, T): S a GPU tensor (N, m) in column order (S.T contiguous), T host (m, m)."""
    import torch

    _, N = sgn_get_dims(ctx)
    T = np.asarray(T, dtype=np.complex128)
    m = T.shape[0]
    if m == 0:
        return _check(ctx, _lib.sgn_deflate_import(ctx, 0, None, None))
    if S.shape != (N, m):
        raise ValueError("S must have shape (N, m)")
    Scols = S.transpose(0, 1).contiguous()  # column j contiguous
    Tf, tp = _hptr(np.asfortranarray(T).ravel(order="F"), m * m, "T")
    st = _lib.sgn_deflate_import(ctx, m, _dptr(Scols, N * m, "S"), tp)
    torch.cuda.synchronize()
    return _check(ctx, st)


def sgn_deflate_export(ctx):
    """Return (S as GPU tensor (N, m), T host (m, m), evals host (m,))."""
    import torch

    _, N = sgn_get_dims(ctx)
    m = _lib.sgn_deflation_size(ctx)
    if m == 0:
        return None, np.zeros((0, 0), complex), np.zeros(0, complex)
    Scols = torch.empty((m, N), dtype=torch.complex128, device="cuda")
    T = np.zeros(m * m, dtype=np.complex128)
    ev = np.zeros(m, dtype=np.complex128)
    _check(ctx, _lib.sgn_deflate_export(ctx, _dptr(Scols), T.ctypes.data_as(C.c_void_p),
                                       ev.ctypes.data_as(C.c_void_p)))
    return Scols.transpose(0, 1), T.reshape(m, m, order="F"), ev


def sgn_deflation_size(ctx):
    return _lib.sgn_deflation_size(ctx)


def sgn_deflation_mode(ctx):
    """SGN_DEFL_NONE, SGN_DEFL_SCHUR or SGN_DEFL_LR."""
    mode = _lib.sgn_deflation_mode(ctx)
    _check(ctx, mode if mode < 0 else SGN_OK)
    return mode


def sgn_set_deflation_filter(ctx, degree, cut=0.0):
    return _check(ctx, _lib.sgn_set_deflation_filter(ctx, int(degree), float(cut)))


def sgn_set_deflation_krylov(ctx, ncv):
    """Krylov subspace size of the deflation eigensolver (0: default rule)."""
    return _check(ctx, _lib.sgn_set_deflation_krylov(ctx, int(ncv)))


def sgn_deflate_lr(ctx, m):
    """LR-deflation pair (right and left critical eigenvectors) computed on the device."""
    return _check(ctx, _lib.sgn_deflate_lr(ctx, int(m)))


def sgn_deflate_lr_import(ctx, R, L, lam):
    """Install R, L (N x m complex128 device tensors, interface layout, L^dag R = I)
    and the eigenvalues lam (m complex, host)."""
    import torch

    _, N = sgn_get_dims(ctx)
    m = int(R.shape[1])
    if R.shape != (N, m) or L.shape != (N, m):
        raise ValueError("R and L must have shape (N, m)")
    Rc = R.t().contiguous()  # column-major N x m = row-major m x N
    Lc = L.t().contiguous()
    lam = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128).ravel())
    if lam.size != m:
        raise ValueError("lam must have m entries")
    torch.cuda.synchronize()  # the library reads Rc, Lc on the context's stream
    return _check(ctx, _lib.sgn_deflate_lr_import(ctx, m, _dptr(Rc, N * m, "R"), _dptr(Lc, N * m, "L"),
                                                  lam.ctypes.data_as(C.c_void_p)))


def sgn_deflate_lr_export(ctx):
    """(R, L, lam): R, L device tensors N x m, lam numpy (m,)."""
    import torch

    _, N = sgn_get_dims(ctx)
    m = sgn_deflation_size(ctx)
    if sgn_deflation_mode(ctx) != SGN_DEFL_LR:
        raise SgnError(SGN_ESTATE, "no LR-deflation pair installed")
    R = torch.empty(m, N, dtype=torch.complex128, device="cuda")
    L = torch.empty(m, N, dtype=torch.complex128, device="cuda")
    lam = np.zeros(m, dtype=np.complex128)
    _check(ctx, _lib.sgn_deflate_lr_export(ctx, _dptr(R, N * m, "R"), _dptr(L, N * m, "L"),
                                           lam.ctypes.data_as(C.c_void_p)))
    return R.t(), L.t(), lam


def sgn_apply(ctx, x, y, tol, kmax):
    """y = sgn(H_w(mu)) x; returns SGN_OK or SGN_ENOCONV (soft)."""
    _, N = sgn_get_dims(ctx)
    st = _lib.sgn_apply(ctx, _dptr(x, N, "x"), _dptr(y, N, "y"), float(tol), int(kmax))
    return _check(ctx, st, soft=(SGN_ENOCONV,))


def sgn_apply_fixed(ctx, x, y, k):
    _, N = sgn_get_dims(ctx)
    return _check(ctx, _lib.sgn_apply_fixed(ctx, _dptr(x, N, "x"), _dptr(y, N, "y"), int(k)))


def sgn_apply_adjoint(ctx, x, y, tol, kmax):
    """y = sgn(H_w(mu))^dag x = sgn(H_w(-mu)) x with the installed LR pair (or
    none); returns SGN_OK or SGN_ENOCONV (soft)."""
    _, N = sgn_get_dims(ctx)
    st = _lib.sgn_apply_adjoint(ctx, _dptr(x, N, "x"), _dptr(y, N, "y"), float(tol), int(kmax))
    return _check(ctx, st, soft=(SGN_ENOCONV,))


def sgn_apply_adjoint_fixed(ctx, x, y, k):
    _, N = sgn_get_dims(ctx)
    return _check(ctx, _lib.sgn_apply_adjoint_fixed(ctx, _dptr(x, N, "x"), _dptr(y, N, "y"), int(k)))


def sgn_overlap_apply_adjoint(ctx, x, y, tol, kmax):
    """y = D_ov(mu)^dag x = x + sgn(H_w(mu))^dag gamma5 x; returns SGN_OK or SGN_ENOCONV (soft)."""
    _, N = sgn_get_dims(ctx)
    st = _lib.sgn_overlap_apply_adjoint(ctx, _dptr(x, N, "x"), _dptr(y, N, "y"), float(tol), int(kmax))
    return _check(ctx, st, soft=(SGN_ENOCONV,))


def sgn_overlap_solve(ctx, b, x, mass, tol, max_iter=500, restart=50, inner_tol=None, inner_kmax=None):
    """x with D(m) x = b, D(m) = (1 - m/2) D_ov(mu) + m, by restarted GMRES
    over sign applies (inner_tol default tol / 100, inner_kmax default
    min(N, 1000)); returns (status, outer steps, true relative residual)."""
    _, N = sgn_get_dims(ctx)
    it, res = C.c_int(0), C.c_double(0.0)
    st = _lib.sgn_overlap_solve(ctx, _dptr(b, N, "b"), _dptr(x, N, "x"), float(mass), float(tol), int(max_iter),
                                int(restart), float(inner_tol if inner_tol is not None else tol / 100.0),
                                int(inner_kmax if inner_kmax is not None else min(N, 1000)), C.byref(it),
                                C.byref(res))
    return _check(ctx, st, soft=(SGN_ENOCONV,)), it.value, res.value


def sgn_apply_batched(ctx, X, Y, tol, kmax):
    """Y[r] = sgn(H_w(mu)) X[r] for the rows of X (nrhs x N complex128 on the
    device); returns (status, [info dict per source])."""
    _, N = sgn_get_dims(ctx)
    nrhs = X.shape[0] if X.dim() == 2 else X.numel() // N
    infos = (sgn_info * nrhs)()
    st = _lib.sgn_apply_batched(ctx, int(nrhs), _dptr(X, nrhs * N, "X"), _dptr(Y, nrhs * N, "Y"), float(tol),
                                int(kmax), infos)
    return _check(ctx, st, soft=(SGN_ENOCONV,)), [infos[r].as_dict() for r in range(nrhs)]


def sgn_overlap_apply(ctx, x, y, tol, kmax):
    """y = D_ov(mu) x = x + gamma5 sgn(H_w(mu)) x; returns SGN_OK or SGN_ENOCONV (soft)."""
    _, N = sgn_get_dims(ctx)
    st = _lib.sgn_overlap_apply(ctx, _dptr(x, N, "x"), _dptr(y, N, "y"), float(tol), int(kmax))
    return _check(ctx, st, soft=(SGN_ENOCONV,))


def sgn_overlap_apply_batched(ctx, X, Y, tol, kmax):
    """Y[r] = D_ov(mu) X[r]; returns (status, [info dict per source])."""
    _, N = sgn_get_dims(ctx)
    nrhs = X.shape[0] if X.dim() == 2 else X.numel() // N
    infos = (sgn_info * nrhs)()
    st = _lib.sgn_overlap_apply_batched(ctx, int(nrhs), _dptr(X, nrhs * N, "X"), _dptr(Y, nrhs * N, "Y"),
                                        float(tol), int(kmax), infos)
    return _check(ctx, st, soft=(SGN_ENOCONV,)), [infos[r].as_dict() for r in range(nrhs)]


def sgn_apply_batched_fixed(ctx, X, Y, k):
    """Exactly k Arnoldi steps per source; returns [info dict per source]."""
    _, N = sgn_get_dims(ctx)
    nrhs = X.shape[0] if X.dim() == 2 else X.numel() // N
    infos = (sgn_info * nrhs)()
    _check(ctx, _lib.sgn_apply_batched_fixed(ctx, int(nrhs), _dptr(X, nrhs * N, "X"), _dptr(Y, nrhs * N, "Y"),
                                             int(k), infos))
    return [infos[r].as_dict() for r in range(nrhs)]


def sgn_apply_adjoint_batched(ctx, X, Y, tol, kmax):
    """Y[r] = sgn(H_w(mu))^dag X[r]; returns (status, [info dict per source])."""
    _, N = sgn_get_dims(ctx)
    nrhs = X.shape[0] if X.dim() == 2 else X.numel() // N
    infos = (sgn_info * nrhs)()
    st = _lib.sgn_apply_adjoint_batched(ctx, int(nrhs), _dptr(X, nrhs * N, "X"), _dptr(Y, nrhs * N, "Y"),
                                        float(tol), int(kmax), infos)
    return _check(ctx, st, soft=(SGN_ENOCONV,)), [infos[r].as_dict() for r in range(nrhs)]


def sgn_apply_adjoint_batched_fixed(ctx, X, Y, k):
    """Exactly k Arnoldi steps per source of the adjoint; returns [info dict per source]."""
    _, N = sgn_get_dims(ctx)
    nrhs = X.shape[0] if X.dim() == 2 else X.numel() // N
    infos = (sgn_info * nrhs)()
    _check(ctx, _lib.sgn_apply_adjoint_batched_fixed(ctx, int(nrhs), _dptr(X, nrhs * N, "X"),
                                                     _dptr(Y, nrhs * N, "Y"), int(k), infos))
    return [infos[r].as_dict() for r in range(nrhs)]


class Session:
    """Serving session on one context (continuous batching; see sgn_session_*
    in include/sgn.h).  Keeps the caller's tensors alive until polled."""

    def __init__(self, ctx, max_slots, kmax):
        self.ctx = ctx
        self.h = _lib.sgn_session_create(ctx, int(max_slots), int(kmax))
        if not self.h:
            raise SgnError(SGN_ESTATE, "sgn_session_create failed: " + (_lib.sgn_last_error(ctx) or b"").decode())
        self._live = {}

    def submit(self, x, y, tol, kmax):
        """Admit a request; returns its handle, or None when no slot is free."""
        _, N = sgn_get_dims(self.ctx)
        req = C.c_int(-1)
        st = _lib.sgn_session_submit(self.h, _dptr(x, N, "x"), _dptr(y, N, "y"), float(tol), int(kmax),
                                     C.byref(req))
        if st == SGN_ENOMEM:
            return None
        _check(self.ctx, st)
        self._live[req.value] = (x, y)
        return req.value

    def step(self, nsteps=1):
        """Advance every occupied slot by up to nsteps steps; returns the
        number of requests finished."""
        st = _lib.sgn_session_step(self.h, int(nsteps))
        if st < 0:
            _check(self.ctx, st)
        return st

    def poll(self, req):
        """None while running, else the request's info dict."""
        info = sgn_info()
        st = _lib.sgn_session_poll(self.h, int(req), C.byref(info))
        if st == 0:
            return None
        self._live.pop(req, None)
        _check(self.ctx, st if st < 0 else SGN_OK)
        return info.as_dict()

    def active(self):
        return _lib.sgn_session_active(self.h)

    def destroy(self):
        if self.h:
            _lib.sgn_session_destroy(self.h)
            self.h = None
            self._live.clear()


def sgn_set_precision(ctx, prec):
    return _check(ctx, _lib.sgn_set_precision(ctx, int(prec)))


def sgn_set_schedule(ctx, k_first, tol):
    return _check(ctx, _lib.sgn_set_schedule(ctx, int(k_first), float(tol)))


def sgn_get_precision(ctx):
    p = _lib.sgn_get_precision(ctx)
    _check(ctx, p if p < 0 else SGN_OK)
    return p


def sgn_set_sign_method(ctx, method):
    return _check(ctx, _lib.sgn_set_sign_method(ctx, int(method)))


def sgn_set_orthogonalization(ctx, mode):
    return _check(ctx, _lib.sgn_set_orthogonalization(ctx, int(mode)))


def sgn_set_block_steps(ctx, s):
    """Block (s-step) Arnoldi process for FP64 applies: s steps per block (0: off)."""
    return _check(ctx, _lib.sgn_set_block_steps(ctx, int(s)))


def sgn_get_block_steps(ctx):
    """(block size, Chebyshev interval half-width in use)."""
    sb, e = C.c_int(), C.c_double()
    _check(ctx, _lib.sgn_get_block_steps(ctx, C.byref(sb), C.byref(e)))
    return sb.value, e.value


def sgn_set_tuning(ctx, update_batch=8, dot_cols=4, update_waves=8):
    """Launch shape of the Arnoldi step's dot and update passes (results are
    bitwise the same for every update_batch and dot_cols; update_waves
    changes them at the rounding level)."""
    return _check(ctx, _lib.sgn_set_tuning(ctx, int(update_batch), int(dot_cols), int(update_waves)))


def sgn_set_step_graphs(ctx, steps):
    """Replay runs of `steps` Arnoldi steps as captured graphs (0: off)."""
    return _check(ctx, _lib.sgn_set_step_graphs(ctx, int(steps)))


def sgn_set_stencil_blocks(ctx, By=0, Bz=0, Bt=0):
    """Stencil walk blocks (0, 0, 0: default; By < 0: natural order); results are bitwise the same."""
    return _check(ctx, _lib.sgn_set_stencil_blocks(ctx, int(By), int(Bz), int(Bt)))


def sgn_get_tuning(ctx):
    ub, cpw, uw = C.c_int(), C.c_int(), C.c_int()
    _check(ctx, _lib.sgn_get_tuning(ctx, C.byref(ub), C.byref(cpw), C.byref(uw)))
    return ub.value, cpw.value, uw.value


def sgn_last_info(ctx):
    info = sgn_info()
    _check(ctx, _lib.sgn_last_info(ctx, C.byref(info)))
    return info.as_dict()


def sgn_footprint_bytes(ctx, kmax, nrhs=1):
    return int(_lib.sgn_footprint_bytes(ctx, int(kmax), int(nrhs)))


def sgn_matvec(ctx, x, y):
    _, N = sgn_get_dims(ctx)
    return _check(ctx, _lib.sgn_matvec(ctx, _dptr(x, N, "x"), _dptr(y, N, "y")))


def sgn_matvec_noalloc(ctx, x, y):
    _, N = sgn_get_dims(ctx)
    return _check(ctx, _lib.sgn_matvec_noalloc(ctx, _dptr(x, N, "x"), _dptr(y, N, "y")))


def sgn_zgemm(ctx, A, B, C):
    """C = A B for GPU complex128 tensors given as column-major matrices: pass
    each matrix M as M.T.contiguous() (shape (cols, rows)); C likewise."""
    K, M = A.shape
    N, K2 = B.shape
    if K2 != K or tuple(C.shape) != (N, M):
        raise ValueError("shapes do not match")
    return _check(ctx, _lib.sgn_zgemm(ctx, M, N, K, _dptr(A, A.numel(), "A"), max(M, 1), _dptr(B, B.numel(), "B"),
                                      max(K, 1), _dptr(C, C.numel(), "C"), max(M, 1)))


def sgn_dense_sign(ctx, A, F):
    """F = sgn(A) for square GPU tensors in column-major order (pass A.T.contiguous())."""
    n = int(round(A.numel() ** 0.5))
    it = C.c_int()
    _check(ctx, _lib.sgn_dense_sign(ctx, n, _dptr(A, n * n, "A"), _dptr(F, n * n, "F"), C.byref(it)))
    return it.value


def sgn_set_profiling(ctx, on):
    return _check(ctx, _lib.sgn_set_profiling(ctx, int(bool(on))))


def sgn_profile_read(ctx):
    arr = (sgn_kstat * 32)()
    n = _lib.sgn_profile_read(ctx, arr, 32)
    _check(ctx, n if n < 0 else SGN_OK)
    return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].ms, "bytes": arr[i].bytes,
                                   "flops": arr[i].flops} for i in range(n)}


def sgn_profile_reset(ctx):
    return _check(ctx, _lib.sgn_profile_reset(ctx))


def sgn_debug_hessenberg(ctx, n, m):
    """(H[:n,:n], c0, beta) of the last apply, host numpy."""
    H = np.zeros(n * n, dtype=np.complex128)
    c0 = np.zeros(max(m, 1), dtype=np.complex128)
    beta = C.c_double()
    _check(ctx, _lib.sgn_debug_hessenberg(ctx, int(n), H.ctypes.data_as(C.c_void_p), c0.ctypes.data_as(C.c_void_p),
                                          C.byref(beta)))
    return H.reshape(n, n, order="F"), c0[:m], beta.value


def sgn_strerror(status):
    return _lib.sgn_strerror(int(status)).decode()


def sgn_last_error(ctx):
    return _lib.sgn_last_error(ctx).decode()


def sgn_create_error():
    return _lib.sgn_create_error().decode()

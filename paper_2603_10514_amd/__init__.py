"""Python binding of libchase.so, the gfx950 library behind include/chase.h.

Argument marshalling only: every step of the solver runs in the HIP library.
Device buffers are torch tensors on the GPU (column-major: stride(0) == 1);
they are passed as raw pointers together with torch's current stream, so the
library's work is ordered after torch's.  Importing this package raises if
libchase.so has not been built (python paper_2603_10514_amd/build.py).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchase.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libchase.so is not built; run `python paper_2603_10514_amd/build.py` "
                      "(the solver has no fallback path)")
lib = ctypes.CDLL(LIB_PATH)

# ----------------------------------------------------------- enums --------
CHASE_OK, CHASE_NOT_CONVERGED = 0, 1
CHASE_EINVAL, CHASE_ENOMEM, CHASE_EDEVICE, CHASE_EINTERNAL, CHASE_EBUSY = -1, -2, -3, -4, -5
REAL64, COMPLEX128 = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
QR_AUTO, QR_CHOL1, QR_CHOL2, QR_SHIFTED, QR_HOUSEHOLDER = 0, 1, 2, 3, 4
QR_NAMES = {1: "chol1", 2: "chol2", 3: "shifted", 4: "householder"}
QR_CODES = {v: k for k, v in QR_NAMES.items()}


class ChaseIterLog(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("locked", ctypes.c_int32),
                ("newly_locked", ctypes.c_int32), ("qr_variant", ctypes.c_int32),
                ("chol_failed", ctypes.c_int32), ("filter_prec", ctypes.c_int32),
                ("deg_min", ctypes.c_int32), ("deg_max", ctypes.c_int32),
                ("matvecs", ctypes.c_int64), ("cond_est", ctypes.c_double),
                ("cond_exact", ctypes.c_double), ("c", ctypes.c_double),
                ("e", ctypes.c_double), ("gamma", ctypes.c_double),
                ("lam1", ctypes.c_double), ("t_filter", ctypes.c_double),
                ("t_qr", ctypes.c_double), ("t_rr", ctypes.c_double),
                ("t_resid", ctypes.c_double), ("qr_fro2", ctypes.c_double),
                ("qr_shift", ctypes.c_double), ("ncols", ctypes.c_int32),
                ("degrees", ctypes.POINTER(ctypes.c_int32)), ("ncols_fp32", ctypes.c_int32)]


LOG_CB = ctypes.CFUNCTYPE(None, ctypes.POINTER(ChaseIterLog), ctypes.c_void_p)
BLOCK_CB = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                            ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p)


class ChaseOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("dtype", ctypes.c_int),
                ("precision", ctypes.c_int), ("deg_opt", ctypes.c_int32),
                ("min_deg", ctypes.c_int32), ("max_deg", ctypes.c_int32),
                ("deg_margin", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("qr_policy", ctypes.c_int), ("est_hi", ctypes.c_double),
                ("est_lo", ctypes.c_double), ("have_bounds", ctypes.c_int32),
                ("lambda_1", ctypes.c_double), ("lambda_l", ctypes.c_double),
                ("lambda_max", ctypes.c_double), ("warm_start", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("lanczos_steps", ctypes.c_int32),
                ("lanczos_nvec", ctypes.c_int32), ("lanczos_v0", ctypes.c_void_p),
                ("inject_chol_fail_iter", ctypes.c_int32),
                ("mixed_switch", ctypes.c_double), ("mixed_buffer32", ctypes.c_int32),
                ("stream", ctypes.c_void_p),
                ("log_cb", LOG_CB), ("log_user", ctypes.c_void_p),
                ("block_cb", BLOCK_CB), ("block_user", ctypes.c_void_p)]


class ChaseInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("matvecs", ctypes.c_int64), ("filter_launches", ctypes.c_int32),
                ("filter_fp32_iters", ctypes.c_int32), ("t_total", ctypes.c_double),
                ("t_filter", ctypes.c_double), ("t_qr", ctypes.c_double),
                ("t_rr", ctypes.c_double), ("t_resid", ctypes.c_double),
                ("t_lanczos", ctypes.c_double), ("lambda_1", ctypes.c_double),
                ("lambda_l", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("matvecs_fp32", ctypes.c_int64), ("t_filter_fp32", ctypes.c_double),
                ("ritz_max", ctypes.c_double), ("filter_launches_fp32", ctypes.c_int32)]


_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_d = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("chase_opts_default", None, [ctypes.POINTER(ChaseOpts)])
_sig("chase_solve", ctypes.c_int, [_p, _i64, _i64, _i32, _i32, _i32, _d, ctypes.POINTER(ChaseOpts),
                                   _dp, _p, _i64, _dp, ctypes.POINTER(ChaseInfo)])
_sig("chase_workspace_bytes", ctypes.c_size_t, [_i64, _i32, _i32, ctypes.c_int, ctypes.c_int])
_sig("chase_handle_create", ctypes.c_int, [_i64, _i32, _i32, ctypes.POINTER(ChaseOpts),
                                           ctypes.POINTER(_p)])
_sig("chase_solve_async", ctypes.c_int, [_p, _p, _i64, _i64, _i32, _i32, _i32, _d,
                                         ctypes.POINTER(ChaseOpts), _dp, _p, _i64, _dp,
                                         ctypes.POINTER(ChaseInfo)])
_sig("chase_handle_query", ctypes.c_int, [_p])
_sig("chase_handle_wait", ctypes.c_int, [_p])
_sig("chase_handle_destroy", None, [_p])
_sig("chase_filter", ctypes.c_int, [ctypes.c_int, ctypes.c_int, _p, _i64, _i64, _p, _i64, _i32,
                                    _ip, _d, _d, _d, _p, _i64, _p])
_sig("chase_filter_noalloc", ctypes.c_int, [ctypes.c_int, _p, _i64, _i64, _p, _i64, _i32, _ip, _d,
                                            _d, _d, _p, _i64, _p])
FILTER_NOALLOC_SCRATCH_BYTES = 64 << 20  # CHASE_FILTER_NOALLOC_SCRATCH_BYTES
_sig("chase_log_cond_estimate", _d, [_d, _i32, _i32, _d, _d, _d])
_sig("chase_select_qr", ctypes.c_int, [_d, _d, _d])
_sig("chase_degrees", None, [_dp, _dp, _i32, _d, _d, _d, _i32, _i32, _i32, _ip])
_sig("chase_qr_factor", ctypes.c_int, [ctypes.c_int, _p, _i64, _i64, _i32, ctypes.c_int, _ip, _dp,
                                       _p])
_sig("chase_rayleigh_ritz", ctypes.c_int, [ctypes.c_int, _p, _i64, _i64, _p, _i64, _i32, _dp,
                                           _p, _i64, _p, _i64, _p])
_sig("chase_residuals", ctypes.c_int, [ctypes.c_int, _p, _i64, _p, _i64, _i64, _i32, _dp, _dp, _p])
_sig("chase_lanczos", ctypes.c_int, [ctypes.c_int, _p, _i64, _i64, _p, _i32, _i32, _i32, _dp, _dp,
                                     _dp, _p])
_sig("chase_lanczos_bounds", ctypes.c_int, [_dp, _dp, _i32, _i32, _i64, _i32, _dp])
_sig("chase_sequence_bounds", ctypes.c_int, [_dp, _d, _dp])
_sig("chase_set_panel_wait_limit", ctypes.c_int, [_i64])
_sig("chase_strerror", ctypes.c_char_p, [ctypes.c_int])
_sig("chase_last_error", ctypes.c_char_p, [])


class ChaseError(RuntimeError):
    def __init__(self, status, where):
        msg = "%s: %s (%s)" % (where, lib.chase_strerror(status).decode(),
                               lib.chase_last_error().decode())
        super().__init__(msg)
        self.status = status


def _check(status, where, allow=(CHASE_OK,)):
    if status not in allow:
        raise ChaseError(status, where)
    return status


# ------------------------------------------------------ marshalling -------
def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return REAL64
    if t.dtype == torch.complex128:
        return COMPLEX128
    raise TypeError("matrices must be float64 or complex128, got %s" % (t.dtype,))


def _colmajor(t, name, allow_symmetric_rowmajor=False):
    """(pointer, leading dimension) of a column-major device matrix."""
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if t.dim() == 1:
        return t.data_ptr(), max(1, t.shape[0])
    if t.stride(0) == 1:
        return t.data_ptr(), max(t.stride(1), t.shape[0])
    if allow_symmetric_rowmajor and t.is_contiguous() and t.shape[0] == t.shape[1]:
        return t.data_ptr(), t.shape[0]
    raise ValueError("%s must be column-major (stride(0) == 1)" % name)


def _hermitian_ptr(H):
    import torch
    # a row-major real symmetric matrix is its own column-major storage
    return _colmajor(H, "H", allow_symmetric_rowmajor=(H.dtype == torch.float64))


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def colmajor_empty(rows, cols, dtype, device):
    """An uninitialised column-major rows x cols device tensor."""
    import torch
    return torch.empty((cols, rows), dtype=dtype, device=device).T


def opts_default(**kw):
    o = ChaseOpts()
    lib.chase_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "qr_policy" and isinstance(v, str):
            v = QR_AUTO if v == "auto" else QR_CODES[v]
        setattr(o, k, v)
    return o


def _info_dict(info):
    return {f: getattr(info, f) for f, _ in ChaseInfo._fields_}


def _log_dict(rec):
    d = {f: getattr(rec, f) for f, _ in ChaseIterLog._fields_ if f != "degrees"}
    d["variant"] = QR_NAMES.get(d["qr_variant"], "?")
    d["degrees"] = [rec.degrees[i] for i in range(rec.ncols)] if rec.degrees else []
    return d


# ----------------------------------------------------------- solve --------
def exact_cond_host(Xptr, N, ld, ncols, cplx):
    """kappa_2 of a device block by an SVD of its host copy (diagnostic)."""
    import torch
    dt = torch.complex128 if cplx else torch.float64
    es = 16 if cplx else 8
    host = torch.empty((ncols, ld), dtype=dt)
    rc = _memcpy_d2h(host.data_ptr(), Xptr, es * ld * ncols)
    if rc != 0:
        return float("nan")
    A = host.numpy().T[:N, :]
    sv = np.linalg.svd(A, compute_uv=False)
    return float(sv[0] / sv[-1]) if sv[-1] > 0 else float("inf")


_HIP = None


def _memcpy_d2h(dst, src, nbytes):
    """hipMemcpy device -> host (the diagnostic copy of exact_cond_host)."""
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.restype = ctypes.c_int
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _HIP.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 2)


def chase_solve(H, nev, nex, degree=20, tol=1e-10, evecs=None, opts=None, stream=None,
                exact_cond=False, **kw):
    """Alg. 1 on the device matrix H.  Returns a dict with status, evals and
    resid (numpy), evecs (the N x (nev+nex) column-major device tensor), info
    and the per-iteration log.  Keyword arguments override chase_opts fields;
    pass evecs with warm_start=1 to start from a given block.  exact_cond adds
    kappa_2 of [Y, filtered] (SVD of a host copy) to every log record."""
    import torch
    N = H.shape[0]
    L = nev + nex
    o = opts if opts is not None else opts_default()
    for k, v in kw.items():
        if k == "qr_policy" and isinstance(v, str):
            v = QR_AUTO if v == "auto" else QR_CODES[v]
        setattr(o, k, v)
    o.dtype = _dtype_code(H)
    hp, ldh = _hermitian_ptr(H)
    if evecs is None:
        evecs = colmajor_empty(N, L, H.dtype, H.device)
    vp, ldv = _colmajor(evecs, "evecs")
    logs = []

    def _cb(rec_ptr, user):
        logs.append(_log_dict(rec_ptr.contents))

    cb = LOG_CB(_cb)
    o.log_cb = cb
    cplx = o.dtype == COMPLEX128
    bcb = BLOCK_CB(lambda X, n, ld, nc, it, user: exact_cond_host(X, n, ld, nc, cplx))
    o.block_cb = bcb if exact_cond else BLOCK_CB()
    o.stream = _stream_ptr(stream).value
    evals = np.zeros(nev)
    resid = np.zeros(nev)
    info = ChaseInfo()
    st = lib.chase_solve(hp, N, ldh, nev, nex, degree, tol, ctypes.byref(o),
                         evals.ctypes.data_as(_dp), vp, ldv, resid.ctypes.data_as(_dp),
                         ctypes.byref(info))
    o.log_cb = LOG_CB()
    o.block_cb = BLOCK_CB()
    _check(st, "chase_solve", (CHASE_OK, CHASE_NOT_CONVERGED))
    return dict(status=st, evals=evals, resid=resid, evecs=evecs, info=_info_dict(info), log=logs)


def chase_workspace_bytes(N, nev, nex, dtype=REAL64, precision=PREC_FP64):
    return int(lib.chase_workspace_bytes(N, nev, nex, dtype, precision))


# ------------------------------------------------------- step calls -------
def chase_filter(H, V, degrees, c, e, gamma, out=None, precision=PREC_FP64, stream=None):
    """Filter every column of V with its own degree (ascending)."""
    N = H.shape[0]
    deg = np.ascontiguousarray(np.asarray(degrees, dtype=np.int32))
    hp, ldh = _hermitian_ptr(H)
    vp, ldv = _colmajor(V, "V")
    if out is None:
        out = colmajor_empty(N, V.shape[1], H.dtype, H.device)
    op, ldo = _colmajor(out, "out")
    st = lib.chase_filter(_dtype_code(H), precision, hp, N, ldh, vp, ldv, int(deg.size),
                          deg.ctypes.data_as(_ip), c, e, gamma, op, ldo, _stream_ptr(stream))
    _check(st, "chase_filter")
    return out


def chase_filter_noalloc(H, V, degrees, c, e, gamma, out, stream=None):
    """chase_filter (FP64) on the library's static scratch: nothing is
    allocated by the library; `out` must be given.  Asynchronous: the
    result is valid once the stream has reached this call's work."""
    N = H.shape[0]
    deg = np.ascontiguousarray(np.asarray(degrees, dtype=np.int32))
    hp, ldh = _hermitian_ptr(H)
    vp, ldv = _colmajor(V, "V")
    op, ldo = _colmajor(out, "out")
    st = lib.chase_filter_noalloc(_dtype_code(H), hp, N, ldh, vp, ldv, int(deg.size),
                                  deg.ctypes.data_as(_ip), c, e, gamma, op, ldo,
                                  _stream_ptr(stream))
    _check(st, "chase_filter_noalloc")
    return out


def chase_log_cond_estimate(theta_next, m_next, m_max, lam1, c, e):
    return float(lib.chase_log_cond_estimate(theta_next, m_next, m_max, lam1, c, e))


def chase_select_qr(est, hi=1e8, lo=20.0):
    return QR_NAMES[int(lib.chase_select_qr(est, hi, lo))]


def chase_degrees(theta, resid, tol, c, e, min_deg=1, max_deg=36, margin=2):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    r = np.ascontiguousarray(resid, dtype=np.float64)
    out = np.zeros(th.size, dtype=np.int32)
    lib.chase_degrees(th.ctypes.data_as(_dp), r.ctypes.data_as(_dp), th.size, tol, c, e,
                      min_deg, max_deg, margin, out.ctypes.data_as(_ip))
    return out


def chase_qr_factor(X, variant, stream=None, return_shift=False):
    """Orthonormalise X in place with one variant; returns chol_failed, or
    (chol_failed, (||X||_F^2, shift)) with return_shift (NaN unless the
    variant is "shifted")."""
    if isinstance(variant, str):
        variant = QR_CODES[variant]
    xp, ldx = _colmajor(X, "X")
    failed = ctypes.c_int32(0)
    sh = np.zeros(2)
    st = lib.chase_qr_factor(_dtype_code(X), xp, X.shape[0], ldx, X.shape[1], variant,
                             ctypes.byref(failed), sh.ctypes.data_as(_dp), _stream_ptr(stream))
    _check(st, "chase_qr_factor")
    if return_shift:
        return bool(failed.value), (float(sh[0]), float(sh[1]))
    return bool(failed.value)


def chase_rayleigh_ritz(H, Q, stream=None):
    N, n = Q.shape
    hp, ldh = _hermitian_ptr(H)
    qp, ldq = _colmajor(Q, "Q")
    V = colmajor_empty(N, n, H.dtype, H.device)
    HV = colmajor_empty(N, n, H.dtype, H.device)
    ritz = np.zeros(n)
    st = lib.chase_rayleigh_ritz(_dtype_code(H), hp, N, ldh, qp, ldq, n, ritz.ctypes.data_as(_dp),
                                 V.data_ptr(), N, HV.data_ptr(), N, _stream_ptr(stream))
    _check(st, "chase_rayleigh_ritz")
    return ritz, V, HV


def chase_residuals(HV, V, ritz, stream=None):
    N, n = V.shape
    hp, ldh = _colmajor(HV, "HV")
    vp, ldv = _colmajor(V, "V")
    th = np.ascontiguousarray(ritz, dtype=np.float64)
    out = np.zeros(n)
    st = lib.chase_residuals(_dtype_code(V), hp, ldh, vp, ldv, N, n, th.ctypes.data_as(_dp),
                             out.ctypes.data_as(_dp), _stream_ptr(stream))
    _check(st, "chase_residuals")
    return out


def chase_lanczos(H, V0, steps, nsearch, stream=None):
    """Lanczos runs from the columns of the device block V0 (N, or N x nvec
    column-major).  Returns (alpha, beta) as nvec x k arrays, k = min(steps,
    N), and the bounds (lambda_1, lambda_l, upper)."""
    N = H.shape[0]
    hp, ldh = _hermitian_ptr(H)
    nvec = 1 if V0.dim() == 1 else V0.shape[1]
    if V0.shape[0] != N or (V0.dim() == 2 and nvec > 1 and V0.stride() != (1, N)):
        raise ValueError("V0 must be N x nvec, column-major with leading dimension N")
    a = np.zeros(nvec * steps)
    b = np.zeros(nvec * steps)
    bounds = np.zeros(3)
    st = lib.chase_lanczos(_dtype_code(H), hp, N, ldh, V0.data_ptr(), nvec, steps, nsearch,
                           a.ctypes.data_as(_dp), b.ctypes.data_as(_dp),
                           bounds.ctypes.data_as(_dp), _stream_ptr(stream))
    _check(st, "chase_lanczos")
    k = min(steps, N)
    return a.reshape(nvec, steps)[:, :k], b.reshape(nvec, steps)[:, :k], tuple(bounds)


def chase_lanczos_bounds(alpha, beta, N, nsearch):
    """Bounds from Lanczos coefficients (nvec x steps arrays; host only)."""
    a = np.ascontiguousarray(np.atleast_2d(alpha), dtype=np.float64)
    b = np.ascontiguousarray(np.atleast_2d(beta), dtype=np.float64)
    if a.shape != b.shape:
        raise ValueError("alpha and beta must have the same shape")
    bounds = np.zeros(3)
    st = lib.chase_lanczos_bounds(a.ctypes.data_as(_dp), b.ctypes.data_as(_dp), a.shape[0],
                                  a.shape[1], N, nsearch, bounds.ctypes.data_as(_dp))
    _check(st, "chase_lanczos_bounds")
    return tuple(bounds)


def chase_sequence_bounds(prev, delta):
    """Bounds for the next problem of a sequence H + D with ||D||_2 <= delta,
    from the previous solve's (lowest Ritz value, largest Ritz value of the
    search space, upper bound)."""
    p = np.ascontiguousarray(prev, dtype=np.float64)
    if p.size != 3:
        raise ValueError("prev must hold three values")
    out = np.zeros(3)
    _check(lib.chase_sequence_bounds(p.ctypes.data_as(_dp), float(delta),
                                     out.ctypes.data_as(_dp)), "chase_sequence_bounds")
    return tuple(float(x) for x in out)


def chase_set_panel_wait_limit(ticks):
    """Test hook: wall-clock ticks a grid-barrier wait (Householder panel,
    one-launch Lanczos) may take before the call reports a device error
    (<= 0: the default)."""
    _check(lib.chase_set_panel_wait_limit(int(ticks)), "chase_set_panel_wait_limit")


# ------------------------------------------------------ async handles -----
class Handle:
    """Owns a chase_handle: its own stream, workspace and worker thread."""

    def __init__(self, N_max, nev_max, nex_max, opts=None):
        o = opts if opts is not None else opts_default()
        h = ctypes.c_void_p()
        _check(lib.chase_handle_create(N_max, nev_max, nex_max, ctypes.byref(o),
                                       ctypes.byref(h)), "chase_handle_create")
        self._h = h
        self._keep = None

    def solve_async(self, H, nev, nex, degree, tol, evecs, opts):
        N = H.shape[0]
        hp, ldh = _hermitian_ptr(H)
        vp, ldv = _colmajor(evecs, "evecs")
        opts.dtype = _dtype_code(H)
        opts.log_cb = LOG_CB()
        opts.block_cb = BLOCK_CB()
        opts.stream = None
        evals = np.zeros(nev)
        resid = np.zeros(nev)
        info = ChaseInfo()
        self._keep = (H, evecs, opts, evals, resid, info)
        _check(lib.chase_solve_async(self._h, hp, N, ldh, nev, nex, degree, tol, ctypes.byref(opts),
                                     evals.ctypes.data_as(_dp), vp, ldv,
                                     resid.ctypes.data_as(_dp), ctypes.byref(info)),
               "chase_solve_async")
        return evals, resid, info

    def query(self):
        return int(lib.chase_handle_query(self._h))

    def wait(self):
        return int(lib.chase_handle_wait(self._h))

    def close(self):
        if self._h:
            lib.chase_handle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""ctypes binding of the hpadi C ABI (include/hpadi.h).

Argument marshalling only: every step of the solver runs in libhpadi.so (host
C++ precomputation and HIP kernels).  torch is used for device memory and the
current stream.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhpadi.so")

HPADI_OK, HPADI_EINVAL, HPADI_ENOTSPD, HPADI_ESINGULAR = 0, -1, -2, -3
HPADI_EINTERVAL, HPADI_ENOCONV, HPADI_EHIP, HPADI_ENOMEM = -4, -5, -6, -7
HPADI_DIRICHLET, HPADI_NEUMANN, HPADI_ROBIN = 0, 1, 2
HPADI_FP64, HPADI_MIXED = 0, 1

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_float_p = ctypes.POINTER(ctypes.c_float)


class hpadi_stats(ctypes.Structure):
    _fields_ = [("J", ctypes.c_int), ("rounds", ctypes.c_int), ("iters", ctypes.c_int),
                ("status", ctypes.c_int), ("interval", ctypes.c_double * 4),
                ("est_rel_err", ctypes.c_double), ("res_rel", ctypes.c_double),
                ("fp32_rounds", ctypes.c_int), ("J_refine", ctypes.c_int), ("t_ms", ctypes.c_double * 3)]


class hpadi_options(ctypes.Structure):
    _fields_ = [("inner_tol", ctypes.c_double), ("max_rounds", ctypes.c_int),
                ("lines_per_block", ctypes.c_int),
                ("fixed_rounds", ctypes.c_int), ("fp32_rounds", ctypes.c_int),
                ("col_lines_per_block", ctypes.c_int), ("refine_tol", ctypes.c_double),
                ("row_lines_per_block", ctypes.c_int)]


class hpadi_krylov_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("precond_calls", ctypes.c_int),
                ("corrections", ctypes.c_int), ("rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("t_ms", ctypes.c_double), ("fallback_iters", ctypes.c_int), ("reserved_i", ctypes.c_int),
                ("reserved", ctypes.c_double * 2)]


# name -> (restype, argtypes), in the order of include/hpadi.h
SIGNATURES = {
    "hpadi_op1d_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         _c_double_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_op1d_create_ex": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            _c_double_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_double, ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_op1d_dims": (ctypes.c_int, [ctypes.c_void_p, _c_int_p, _c_int_p]),
    "hpadi_op1d_export": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, _c_double_p, _c_double_p]),
    "hpadi_op1d_destroy": (None, [ctypes.c_void_p]),
    "hpadi_interval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, _c_double_p]),
    "hpadi_shifts": (ctypes.c_int, [_c_double_p, ctypes.c_double, ctypes.c_int, _c_int_p, _c_double_p,
                                    _c_double_p, ctypes.c_int]),
    "hpadi_plan_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, _c_double_p, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_plan_create_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int, _c_double_p, ctypes.c_void_p,
                                            ctypes.POINTER(hpadi_options), ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_plan_create_general": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _c_double_p, ctypes.c_double,
                                                 ctypes.c_int, _c_double_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_plan_info": (ctypes.c_int, [ctypes.c_void_p, _c_int_p, _c_double_p, _c_double_p, _c_double_p]),
    "hpadi_plan_export_factor": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_double_p,
                                                ctypes.c_size_t]),
    "hpadi_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]),
    "hpadi_load_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_int]),
    "hpadi_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.POINTER(hpadi_stats)]),
    "hpadi_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]),
    "hpadi_plan_destroy": (None, [ctypes.c_void_p]),
    "hpadi_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_void_p), _c_double_p, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_void_p), _c_int_p, ctypes.POINTER(ctypes.c_void_p),
                                          _c_int_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_batch_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(hpadi_stats), _c_int_p]),
    "hpadi_batch_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_int_p, _c_int_p, _c_int_p]),
    "hpadi_batch_destroy": (None, [ctypes.c_void_p]),
    "hpadi_varcoef_grid": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, _c_double_p, ctypes.c_int]),
    "hpadi_varcoef_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_varcoef_create_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                               ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_varcoef_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_int]),
    "hpadi_varcoef_destroy": (None, [ctypes.c_void_p]),
    "hpadi_net_num_params": (ctypes.c_int, []),
    "hpadi_net_create": (ctypes.c_int, [_c_float_p, ctypes.c_ulonglong, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_net_get_params": (ctypes.c_int, [ctypes.c_void_p, _c_float_p]),
    "hpadi_net_set_params": (ctypes.c_int, [ctypes.c_void_p, _c_float_p]),
    "hpadi_net_set_damping": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "hpadi_net_set_period": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "hpadi_net_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_void_p]),
    "hpadi_net_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_double), _c_float_p]),
    "hpadi_net_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_ulonglong, _c_float_p]),
    "hpadi_net_pairs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_ulonglong, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, _c_int_p]),
    "hpadi_net_destroy": (None, [ctypes.c_void_p]),
    "hpadi_fcg_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, _c_double_p, ctypes.c_int, ctypes.POINTER(hpadi_krylov_stats)]),
    "hpadi_grid": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, ctypes.c_int]),
    "hpadi_transform_export": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_double_p, ctypes.c_int]),
    "hpadi_transform_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_values_to_legendre": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                                ctypes.c_int]),
    "hpadi_legendre_to_values": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                                ctypes.c_int]),
    "hpadi_q_to_values": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_int]),
    "hpadi_transform_destroy": (None, [ctypes.c_void_p]),
    "hpadi_burgers_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_void_p)]),
    "hpadi_burgers_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p]),
    "hpadi_burgers_destroy": (None, [ctypes.c_void_p]),
    "hpadi_plan_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "hpadi_plan_timing_read": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, _c_double_p, _c_int_p]),
    "hpadi_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libhpadi.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2402_11299_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class HpadiError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().hpadi_strerror(status).decode()
        super().__init__(f"{where}: {msg} ({status})")


def check(status: int, where: str) -> None:
    if status != HPADI_OK:
        raise HpadiError(status, where)


def _dptr(arr):
    import numpy as np
    assert arr.dtype == np.float64 and arr.flags["C_CONTIGUOUS"]
    return arr.ctypes.data_as(_c_double_p)


# --------------------------------------------------------------------------
# Thin wrappers with the C names.
# --------------------------------------------------------------------------

def hpadi_op1d_create(n, p, a=0.0, b=1.0, breaks=None, bc=HPADI_DIRICHLET):
    import numpy as np
    h = ctypes.c_void_p()
    br = None
    if breaks is not None:
        br = np.ascontiguousarray(breaks, dtype=np.float64)
    check(lib().hpadi_op1d_create(int(n), int(p), float(a), float(b), _dptr(br) if br is not None else None,
                                  int(bc), ctypes.byref(h)), "hpadi_op1d_create")
    return h


def hpadi_op1d_create_ex(n, p, a=0.0, b=1.0, breaks=None, bc_left=HPADI_DIRICHLET, bc_right=HPADI_DIRICHLET,
                         alpha_left=0.0, alpha_right=0.0):
    import numpy as np
    h = ctypes.c_void_p()
    br = None
    if breaks is not None:
        br = np.ascontiguousarray(breaks, dtype=np.float64)
    check(lib().hpadi_op1d_create_ex(int(n), int(p), float(a), float(b), _dptr(br) if br is not None else None,
                                     int(bc_left), int(bc_right), float(alpha_left), float(alpha_right),
                                     ctypes.byref(h)), "hpadi_op1d_create_ex")
    return h


def hpadi_op1d_dims(op):
    N, L = ctypes.c_int(), ctypes.c_int()
    check(lib().hpadi_op1d_dims(op, ctypes.byref(N), ctypes.byref(L)), "hpadi_op1d_dims")
    return N.value, L.value


def hpadi_op1d_export(op):
    import numpy as np
    N, L = hpadi_op1d_dims(op)
    K, M, T = np.zeros((N, N)), np.zeros((N, N)), np.zeros((N, L))
    check(lib().hpadi_op1d_export(op, _dptr(K), _dptr(M), _dptr(T)), "hpadi_op1d_export")
    return K, M, T


def hpadi_op1d_destroy(op):
    lib().hpadi_op1d_destroy(op)


def hpadi_interval(op, omega2):
    out = (ctypes.c_double * 2)()
    check(lib().hpadi_interval(op, float(omega2), out), "hpadi_interval")
    return out[0], out[1]


def hpadi_shifts(iv, tol, J=0, maxJ=512):
    iv_c = (ctypes.c_double * 4)(*[float(v) for v in iv])
    Jc = ctypes.c_int()
    p = (ctypes.c_double * maxJ)()
    q = (ctypes.c_double * maxJ)()
    check(lib().hpadi_shifts(iv_c, float(tol), int(J), ctypes.byref(Jc), p, q, maxJ), "hpadi_shifts")
    return Jc.value, list(p[:Jc.value]), list(q[:Jc.value])


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def hpadi_plan_create(x, y, omega2, tol, precision=HPADI_FP64, interval=None, stream=None, options=None):
    h = ctypes.c_void_p()
    iv = (ctypes.c_double * 4)(*[float(v) for v in interval]) if interval is not None else None
    if options is None:
        st = lib().hpadi_plan_create(x, y, float(omega2), float(tol), int(precision), iv,
                                     _stream_handle(stream), ctypes.byref(h))
    else:
        st = lib().hpadi_plan_create_ex(x, y, float(omega2), float(tol), int(precision), iv,
                                        _stream_handle(stream), ctypes.byref(options), ctypes.byref(h))
    check(st, "hpadi_plan_create")
    return h


def hpadi_plan_create_general(x, y, coef, tol, precision=HPADI_FP64, interval=None, stream=None, options=None):
    h = ctypes.c_void_p()
    cf = (ctypes.c_double * 4)(*[float(v) for v in coef])
    iv = (ctypes.c_double * 4)(*[float(v) for v in interval]) if interval is not None else None
    check(lib().hpadi_plan_create_general(x, y, cf, float(tol), int(precision), iv, _stream_handle(stream),
                                          ctypes.byref(options) if options is not None else None,
                                          ctypes.byref(h)), "hpadi_plan_create_general")
    return h


def hpadi_plan_info(plan, maxJ=512):
    J = ctypes.c_int()
    p = (ctypes.c_double * maxJ)()
    q = (ctypes.c_double * maxJ)()
    iv = (ctypes.c_double * 4)()
    check(lib().hpadi_plan_info(plan, ctypes.byref(J), None, None, iv), "hpadi_plan_info")
    if J.value > maxJ:
        raise ValueError("too many shifts")
    check(lib().hpadi_plan_info(plan, ctypes.byref(J), p, q, iv), "hpadi_plan_info")
    return J.value, list(p[:J.value]), list(q[:J.value]), list(iv)


def hpadi_plan_export_factor(plan, j, axis, length):
    import numpy as np
    buf = np.zeros(length)
    check(lib().hpadi_plan_export_factor(plan, int(j), int(axis), _dptr(buf), buf.size),
          "hpadi_plan_export_factor")
    return buf


def _tptr(t, dtype_name="float64"):
    import torch
    if not t.is_cuda or t.dtype != getattr(torch, dtype_name) or t.stride(1) != 1:
        raise ValueError("expected a row-major CUDA float64 tensor")
    return ctypes.c_void_p(t.data_ptr()), int(t.stride(0))


def hpadi_load(plan, F, G):
    fp, ldf = _tptr(F)
    gp, ldg = _tptr(G)
    check(lib().hpadi_load(plan, fp, ldf, gp, ldg), "hpadi_load")


def hpadi_load_noalloc(plan, F, G):
    fp, ldf = _tptr(F)
    gp, ldg = _tptr(G)
    check(lib().hpadi_load_noalloc(plan, fp, ldf, gp, ldg), "hpadi_load_noalloc")


def hpadi_solve(plan, G, U, raise_on_noconv=True):
    gp, ldg = _tptr(G)
    up, ldu = _tptr(U)
    st = hpadi_stats()
    rc = lib().hpadi_solve(plan, gp, ldg, up, ldu, ctypes.byref(st))
    if rc != HPADI_OK and (raise_on_noconv or rc != HPADI_ENOCONV):
        raise HpadiError(rc, "hpadi_solve")
    return st


def hpadi_apply(plan, U, Y):
    up, ldu = _tptr(U)
    yp, ldy = _tptr(Y)
    check(lib().hpadi_apply(plan, up, ldu, yp, ldy), "hpadi_apply")


def hpadi_plan_destroy(plan):
    lib().hpadi_plan_destroy(plan)


def hpadi_varcoef_grid(op, n, p):
    import numpy as np
    q = p + 2
    x = np.zeros(n * q)
    w = np.zeros(n * q)
    check(lib().hpadi_varcoef_grid(op, _dptr(x), _dptr(w), n * q), "hpadi_varcoef_grid")
    return x, w


def hpadi_varcoef_create_ex(x, y, a, c, stream=None):
    ap, lda = _tptr(a) if a is not None else (None, 0)
    cp, ldc = _tptr(c) if c is not None else (None, 0)
    h = ctypes.c_void_p()
    check(lib().hpadi_varcoef_create_ex(x, y, ap, lda, cp, ldc, _stream_handle(stream), ctypes.byref(h)),
          "hpadi_varcoef_create_ex")
    return h


def hpadi_varcoef_create(x, y, a, stream=None):
    ap, lda = _tptr(a)
    h = ctypes.c_void_p()
    check(lib().hpadi_varcoef_create(x, y, ap, lda, _stream_handle(stream), ctypes.byref(h)),
          "hpadi_varcoef_create")
    return h


def hpadi_varcoef_apply(vc, U, Y):
    up, ldu = _tptr(U)
    yp, ldy = _tptr(Y)
    check(lib().hpadi_varcoef_apply(vc, up, ldu, yp, ldy), "hpadi_varcoef_apply")


def hpadi_varcoef_destroy(vc):
    lib().hpadi_varcoef_destroy(vc)


def hpadi_fcg_solve(vc, precond, b, x, tol, maxit, truncation, hist_len=0, raise_on_noconv=True, net=None):
    import numpy as np
    bp, ldb = _tptr(b)
    xp, ldx = _tptr(x)
    hist = np.zeros(max(hist_len, 1))
    st = hpadi_krylov_stats()
    rc = lib().hpadi_fcg_solve(vc, precond, net, bp, ldb, xp, ldx, float(tol), int(maxit), int(truncation),
                               _dptr(hist) if hist_len > 0 else None, int(hist_len), ctypes.byref(st))
    if rc != HPADI_OK and (raise_on_noconv or rc != HPADI_ENOCONV):
        raise HpadiError(rc, "hpadi_fcg_solve")
    return st, hist[:min(st.iters + 1, hist_len)] if hist_len > 0 else None


def hpadi_grid(op, n, p):
    import numpy as np
    x = np.zeros(n * (p + 1))
    check(lib().hpadi_grid(op, _dptr(x), x.size), "hpadi_grid")
    return x


def hpadi_transform_export(p, which):
    import numpy as np
    buf = np.zeros((p + 1) * (p + 1))
    check(lib().hpadi_transform_export(int(p), int(which), _dptr(buf), buf.size), "hpadi_transform_export")
    return buf.reshape(p + 1, p + 1)


def hpadi_transform_create(x, y, stream=None):
    h = ctypes.c_void_p()
    check(lib().hpadi_transform_create(x, y, _stream_handle(stream), ctypes.byref(h)), "hpadi_transform_create")
    return h


def hpadi_values_to_legendre(t, V, F):
    vp, ldv = _tptr(V)
    fp, ldf = _tptr(F)
    check(lib().hpadi_values_to_legendre(t, vp, ldv, fp, ldf), "hpadi_values_to_legendre")


def hpadi_legendre_to_values(t, F, V):
    fp, ldf = _tptr(F)
    vp, ldv = _tptr(V)
    check(lib().hpadi_legendre_to_values(t, fp, ldf, vp, ldv), "hpadi_legendre_to_values")


def hpadi_q_to_values(t, deriv_x, U, V):
    up, ldu = _tptr(U)
    vp, ldv = _tptr(V)
    check(lib().hpadi_q_to_values(t, int(deriv_x), up, ldu, vp, ldv), "hpadi_q_to_values")


def hpadi_transform_destroy(t):
    lib().hpadi_transform_destroy(t)


def hpadi_burgers_create(x, y, eps, dt, tol, precision=HPADI_FP64, options=None, stream=None):
    h = ctypes.c_void_p()
    check(lib().hpadi_burgers_create(x, y, float(eps), float(dt), float(tol), int(precision),
                                     ctypes.byref(options) if options is not None else None,
                                     _stream_handle(stream), ctypes.byref(h)), "hpadi_burgers_create")
    return h


def hpadi_burgers_step(b, F, nsteps, raise_on_noconv=True):
    fp, ldf = _tptr(F)
    st = hpadi_stats()
    rc = lib().hpadi_burgers_step(b, fp, ldf, int(nsteps), ctypes.byref(st))
    if rc != HPADI_OK and (raise_on_noconv or rc != HPADI_ENOCONV):
        raise HpadiError(rc, "hpadi_burgers_step")
    return st


def hpadi_burgers_destroy(b):
    lib().hpadi_burgers_destroy(b)


def hpadi_plan_timing(plan, enable):
    check(lib().hpadi_plan_timing(plan, int(bool(enable))), "hpadi_plan_timing")


def hpadi_plan_timing_read(plan):
    ms = (ctypes.c_double * 6)()
    by = (ctypes.c_double * 6)()
    ct = (ctypes.c_int * 6)()
    check(lib().hpadi_plan_timing_read(plan, ms, by, ct), "hpadi_plan_timing_read")
    return list(ms), list(by), list(ct)


def hpadi_strerror(status):
    return lib().hpadi_strerror(int(status)).decode()


# --------------------------------------------------------------------------
# Small object layer.
# --------------------------------------------------------------------------

_BC_CODES = {"dirichlet": HPADI_DIRICHLET, "neumann": HPADI_NEUMANN, "robin": HPADI_ROBIN}


class Op1D:
    """A 1D discretisation handle (mesh, degree, boundary conditions).  bc: one kind for both
    ends ("dirichlet" or "neumann") or a pair (left, right) of "dirichlet", "neumann",
    "robin"; alpha: the Robin coefficients of the two ends."""

    def __init__(self, n, p, a=0.0, b=1.0, bc="dirichlet", breaks=None, alpha=(0.0, 0.0)):
        self.n, self.p, self.a, self.b = n, p, a, b
        self.bc = bc
        if isinstance(bc, str):
            code = HPADI_DIRICHLET if bc == "dirichlet" else HPADI_NEUMANN
            self.handle = hpadi_op1d_create(n, p, a, b, breaks, code)
        else:
            self.handle = hpadi_op1d_create_ex(n, p, a, b, breaks, _BC_CODES[bc[0]], _BC_CODES[bc[1]],
                                               alpha[0], alpha[1])
        self.N, self.Nleg = hpadi_op1d_dims(self.handle)

    def close(self):
        if self.handle is not None:
            hpadi_op1d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Factorised ADI plan on the GPU (Alg. 2 precomputation)."""

    def __init__(self, x: Op1D, y: Op1D, omega2, tol, precision="fp64", interval=None, stream=None,
                 options=None, coef=None):
        """coef = (kx, sx, ky, sy): the general operator (kx K_x + sx M_x) U M_y + M_x U (ky K_y + sy M_y)
        (omega2 is then ignored); default the screened Poisson operator with omega2."""
        self.x, self.y = x, y
        self.precision = precision
        code = HPADI_FP64 if precision == "fp64" else HPADI_MIXED
        if coef is None:
            self.handle = hpadi_plan_create(x.handle, y.handle, omega2, tol, code, interval, stream, options)
        else:
            self.handle = hpadi_plan_create_general(x.handle, y.handle, coef, tol, code, interval, stream, options)
        self.J, self.p, self.q, self.interval = hpadi_plan_info(self.handle)

    def load(self, F):
        import torch
        if tuple(F.shape) != (self.x.Nleg, self.y.Nleg):
            raise ValueError(f"F must be {self.x.Nleg} x {self.y.Nleg}")
        G = torch.empty((self.x.N, self.y.N), dtype=torch.float64, device=F.device)
        hpadi_load(self.handle, F, G)
        return G

    def solve(self, G, U=None, raise_on_noconv=True):
        import torch
        if tuple(G.shape) != (self.x.N, self.y.N) or (U is not None and tuple(U.shape) != tuple(G.shape)):
            raise ValueError(f"G and U must be {self.x.N} x {self.y.N}")
        if U is None:
            U = torch.empty((self.x.N, self.y.N), dtype=torch.float64, device=G.device)
        st = hpadi_solve(self.handle, G, U, raise_on_noconv)
        return U, st

    def apply(self, U):
        import torch
        if tuple(U.shape) != (self.x.N, self.y.N):
            raise ValueError(f"U must be {self.x.N} x {self.y.N}")
        Y = torch.empty_like(U)
        hpadi_apply(self.handle, U, Y)
        return Y

    def close(self):
        if self.handle is not None:
            hpadi_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VarCoef:
    """Operator -div(a grad u) + c u on the bases of x and y (a = None: a = 1; c = None:
    no potential term)."""

    def __init__(self, x: Op1D, y: Op1D, a, stream=None, c=None):
        self.x, self.y = x, y
        qx, qy = x.p + 2, y.p + 2
        for name, f in (("a", a), ("c", c)):
            if f is not None and tuple(f.shape) != (x.n * qx, y.n * qy):
                raise ValueError(f"{name} must be {x.n * qx} x {y.n * qy} (Gauss grid)")
        if c is None and a is not None:
            self.handle = hpadi_varcoef_create(x.handle, y.handle, a, stream)
        else:
            self.handle = hpadi_varcoef_create_ex(x.handle, y.handle, a, c, stream)

    @staticmethod
    def grid(op: Op1D):
        return hpadi_varcoef_grid(op.handle, op.n, op.p)

    def apply(self, U):
        import torch
        if tuple(U.shape) != (self.x.N, self.y.N):
            raise ValueError(f"U must be {self.x.N} x {self.y.N}")
        Y = torch.empty_like(U)
        hpadi_varcoef_apply(self.handle, U, Y)
        return Y

    def solve(self, b, precond: "Plan" = None, tol=1e-10, maxit=500, truncation=1, hist_len=0,
              raise_on_noconv=True, net: "Net" = None):
        import torch
        if tuple(b.shape) != (self.x.N, self.y.N):
            raise ValueError(f"b must be {self.x.N} x {self.y.N}")
        x = torch.empty_like(b)
        st, hist = hpadi_fcg_solve(self.handle, precond.handle if precond is not None else None, b, x, tol,
                                   maxit, truncation, hist_len, raise_on_noconv,
                                   net.handle if net is not None else None)
        return x, st, hist

    def pairs(self, precond: "Plan", b, xstar, crop, crops_per_iter, cap, tol=1e-10, max_iters=500, seed=0):
        """Training crops from the preconditioned CG iterates (see hpadi_net_pairs)."""
        import torch
        dev = b.device
        X = torch.empty((cap, crop, crop, 3), dtype=torch.float32, device=dev)
        ZN = torch.empty((cap, crop, crop), dtype=torch.float32, device=dev)
        T = torch.empty_like(ZN)
        W = torch.empty_like(ZN)
        bp, ldb = _tptr(b)
        xp, ldx = _tptr(xstar)
        cnt = ctypes.c_int()
        check(lib().hpadi_net_pairs(self.handle, precond.handle, bp, ldb, xp, ldx, float(tol), int(max_iters),
                                    int(crop), int(crops_per_iter), ctypes.c_ulonglong(seed),
                                    ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(ZN.data_ptr()),
                                    ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(W.data_ptr()), int(cap),
                                    ctypes.byref(cnt)), "hpadi_net_pairs")
        k = cnt.value
        return X[:k], ZN[:k], T[:k], W[:k]

    def close(self):
        if getattr(self, "handle", None) is not None:
            hpadi_varcoef_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _fptr_dev(t):
    import torch
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA float32 tensor")
    return ctypes.c_void_p(t.data_ptr())


class Net:
    """Learned correction network (BF16 matrix-core kernels, FP32 parameters)."""

    def __init__(self, params=None, seed=0, stream=None):
        import numpy as np
        h = ctypes.c_void_p()
        self.nparams = lib().hpadi_net_num_params()
        if params is not None:
            arr = np.ascontiguousarray(params, dtype=np.float32)
            if arr.size != self.nparams:
                raise ValueError(f"expected {self.nparams} parameters")
            pp = arr.ctypes.data_as(_c_float_p)
        else:
            pp = None
        check(lib().hpadi_net_create(pp, ctypes.c_ulonglong(seed), _stream_handle(stream), ctypes.byref(h)),
              "hpadi_net_create")
        self.handle = h

    def get_params(self):
        import numpy as np
        out = np.zeros(self.nparams, dtype=np.float32)
        check(lib().hpadi_net_get_params(self.handle, out.ctypes.data_as(_c_float_p)), "hpadi_net_get_params")
        return out

    def set_params(self, params):
        import numpy as np
        arr = np.ascontiguousarray(params, dtype=np.float32)
        check(lib().hpadi_net_set_params(self.handle, arr.ctypes.data_as(_c_float_p)), "hpadi_net_set_params")

    def set_damping(self, omega):
        """0: energy-optimal combination of z and the correction; omega > 0: z + omega c."""
        check(lib().hpadi_net_set_damping(self.handle, float(omega)), "hpadi_net_set_damping")

    def set_period(self, period):
        """Correct at every period-th Krylov iteration only (1: every iteration)."""
        check(lib().hpadi_net_set_period(self.handle, int(period)), "hpadi_net_set_period")

    def forward(self, x):
        import torch
        B, H, W, C = x.shape
        if C != 3:
            raise ValueError("x must be B x H x W x 3")
        out = torch.empty((B, H, W), dtype=torch.float32, device=x.device)
        check(lib().hpadi_net_forward(self.handle, _fptr_dev(x), B, H, W, _fptr_dev(out)), "hpadi_net_forward")
        return out

    def loss_grad(self, x, zn, t, w):
        import numpy as np
        B, H, W, _ = x.shape
        loss = ctypes.c_double()
        g = np.zeros(self.nparams, dtype=np.float32)
        check(lib().hpadi_net_loss_grad(self.handle, _fptr_dev(x), _fptr_dev(zn), _fptr_dev(t), _fptr_dev(w), B, H,
                                        W, ctypes.byref(loss), g.ctypes.data_as(_c_float_p)), "hpadi_net_loss_grad")
        return loss.value, g

    def train(self, X, ZN, T, W, batch, steps, lr, seed=0):
        import numpy as np
        n, c = X.shape[0], X.shape[1]
        hist = np.zeros(max(steps, 1), dtype=np.float32)
        check(lib().hpadi_net_train(self.handle, _fptr_dev(X), _fptr_dev(ZN), _fptr_dev(T), _fptr_dev(W), n, c,
                                    int(batch), int(steps), float(lr), ctypes.c_ulonglong(seed),
                                    hist.ctypes.data_as(_c_float_p)), "hpadi_net_train")
        return hist[:steps]

    def close(self):
        if getattr(self, "handle", None) is not None:
            lib().hpadi_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent solves replayed as one graph (hpadi_batch_*).  problems: list of
    (Op1D x, Op1D y, omega2); G, U: lists of FP64 CUDA tensors bound to the graph."""

    def __init__(self, problems, tol, G, U, autotune=True, nstreams=0, stream=None):
        n = len(problems)
        if len(G) != n or len(U) != n:
            raise ValueError("one G and one U per problem")
        self.problems, self.G, self.U = problems, G, U
        VP = ctypes.c_void_p * n
        xs = VP(*[pr[0].handle.value if hasattr(pr[0].handle, "value") else pr[0].handle for pr in problems])
        ys = VP(*[pr[1].handle.value if hasattr(pr[1].handle, "value") else pr[1].handle for pr in problems])
        w2 = (ctypes.c_double * n)(*[float(pr[2]) for pr in problems])
        gp, ldg, up, ldu = [], [], [], []
        for g, u, pr in zip(G, U, problems):
            if tuple(g.shape) != (pr[0].N, pr[1].N) or tuple(u.shape) != tuple(g.shape):
                raise ValueError("G and U must be N_x x N_y")
            a, la = _tptr(g)
            b, lb = _tptr(u)
            gp.append(a.value)
            ldg.append(la)
            up.append(b.value)
            ldu.append(lb)
        self._keep = (xs, ys, w2, VP(*gp), (ctypes.c_int * n)(*ldg), VP(*up), (ctypes.c_int * n)(*ldu))
        h = ctypes.c_void_p()
        check(lib().hpadi_batch_create(n, xs, ys, w2, float(tol), self._keep[3], self._keep[4], self._keep[5],
                                       self._keep[6], int(bool(autotune)), int(nstreams), _stream_handle(stream),
                                       ctypes.byref(h)), "hpadi_batch_create")
        self.handle = h
        self.count = n

    def solve(self, raise_on_noconv=True):
        st = (hpadi_stats * self.count)()
        extra = ctypes.c_int()
        rc = lib().hpadi_batch_solve(self.handle, st, ctypes.byref(extra))
        if rc != HPADI_OK and (raise_on_noconv or rc != HPADI_ENOCONV):
            raise HpadiError(rc, "hpadi_batch_solve")
        return list(st), extra.value

    def info(self, i):
        lw, J, si = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().hpadi_batch_info(self.handle, int(i), ctypes.byref(lw), ctypes.byref(J), ctypes.byref(si)),
              "hpadi_batch_info")
        return lw.value, J.value, si.value

    def close(self):
        if getattr(self, "handle", None) is not None:
            lib().hpadi_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Transform:
    """Grid transforms of Sec. 6 on the GPU: grid values <-> piecewise Legendre
    coefficients, and hat+bubble coefficients -> grid values of u or du/dx."""

    def __init__(self, x: Op1D, y: Op1D, stream=None):
        self.x, self.y = x, y
        self.handle = hpadi_transform_create(x.handle, y.handle, stream)

    @staticmethod
    def grid(op: Op1D):
        return hpadi_grid(op.handle, op.n, op.p)

    def _out(self, rows, cols, like):
        import torch
        return torch.empty((rows, cols), dtype=torch.float64, device=like.device)

    def values_to_legendre(self, V):
        if tuple(V.shape) != (self.x.Nleg, self.y.Nleg):
            raise ValueError(f"V must be {self.x.Nleg} x {self.y.Nleg}")
        F = self._out(self.x.Nleg, self.y.Nleg, V)
        hpadi_values_to_legendre(self.handle, V, F)
        return F

    def legendre_to_values(self, F):
        if tuple(F.shape) != (self.x.Nleg, self.y.Nleg):
            raise ValueError(f"F must be {self.x.Nleg} x {self.y.Nleg}")
        V = self._out(self.x.Nleg, self.y.Nleg, F)
        hpadi_legendre_to_values(self.handle, F, V)
        return V

    def q_to_values(self, U, deriv_x=False):
        if tuple(U.shape) != (self.x.N, self.y.N):
            raise ValueError(f"U must be {self.x.N} x {self.y.N}")
        V = self._out(self.x.Nleg, self.y.Nleg, U)
        hpadi_q_to_values(self.handle, deriv_x, U, V)
        return V

    def close(self):
        if getattr(self, "handle", None) is not None:
            hpadi_transform_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Burgers:
    """The IMEX time-stepper of Sec. 6 for u_t + u u_x = eps Laplace(u)."""

    def __init__(self, x: Op1D, y: Op1D, eps, dt, tol=1e-12, precision="fp64", options=None, stream=None):
        self.x, self.y = x, y
        self.eps, self.dt = eps, dt
        code = HPADI_FP64 if precision == "fp64" else HPADI_MIXED
        self.handle = hpadi_burgers_create(x.handle, y.handle, eps, dt, tol, code, options, stream)

    def step(self, F, nsteps=1, raise_on_noconv=True):
        """Advance F (Nleg_x x Nleg_y Legendre coefficients, CUDA float64) in place."""
        if tuple(F.shape) != (self.x.Nleg, self.y.Nleg):
            raise ValueError(f"F must be {self.x.Nleg} x {self.y.Nleg}")
        return hpadi_burgers_step(self.handle, F, nsteps, raise_on_noconv)

    def close(self):
        if getattr(self, "handle", None) is not None:
            hpadi_burgers_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""ctypes binding of libxo.so (argument marshalling only).

Every compute step runs in the library's HIP kernels. PyTorch provides device
memory and the current stream. If the library is missing the calls raise: there
is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxo.so")

XO_OK, XO_ERR_ARG, XO_ERR_ALLOC, XO_ERR_HIP, XO_ERR_NOTPD, XO_ERR_UNSUPPORTED, XO_ERR_SINGULAR = range(7)
XO_FP64, XO_FP32, XO_BF16X3, XO_BF16 = 0, 1, 2, 3
XO_EPS_SYM, XO_EPS_NONSYM, XO_EPS_LU_FALLBACK = 0, 1, 2

PREC = {"fp64": XO_FP64, "fp32": XO_FP32, "bf16x3": XO_BF16X3, "bf16": XO_BF16}
ERRNAME = {1: "XO_ERR_ARG", 2: "XO_ERR_ALLOC", 3: "XO_ERR_HIP", 4: "XO_ERR_NOTPD", 5: "XO_ERR_UNSUPPORTED", 6: "XO_ERR_SINGULAR"}

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


class RhoArgs(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3), ("bvec", C.c_double * 9), ("prec", C.c_int),
        ("npw_c", C.c_int), ("mill_c", _i32p), ("nc", C.c_int), ("coef_c", C.c_void_p),
        ("e_c", C.c_void_p), ("kcart", C.c_double * 3),
        ("npw_v", C.c_int), ("mill_v", _i32p), ("nv", C.c_int), ("coef_v", C.c_void_p),
        ("e_v", C.c_void_p), ("g0", C.c_int * 3),
        ("ng", C.c_int), ("mill_g", _i32p), ("q0", C.c_int), ("qhat", C.c_double * 3),
        ("rho", C.c_void_p), ("dE", C.c_void_p),
    ]


class Chi0Args(C.Structure):
    _fields_ = [
        ("nt", C.c_int), ("ng", C.c_int), ("nw", C.c_int), ("prec", C.c_int),
        ("rho", C.c_void_p), ("dE", C.c_void_p), ("w", _f64p), ("pref", C.c_double),
        ("accumulate", C.c_int), ("check_dE", C.c_int), ("chi0", C.c_void_p),
    ]


class EpsArgs(C.Structure):
    _fields_ = [
        ("ng", C.c_int), ("nw", C.c_int), ("qpg", _f64p), ("chi0", C.c_void_p),
        ("flags", C.c_int), ("out", C.c_void_p), ("info", C.c_void_p),
    ]


class TailArgs(C.Structure):
    _fields_ = [
        ("chi_t", C.c_void_p), ("chi_h", C.c_void_p), ("chi_f", C.c_void_p), ("qpg", _f64p),
        ("mill_g", C.POINTER(C.c_int32)), ("bvec", _f64p), ("w", _f64p), ("ng", C.c_int), ("nw", C.c_int),
        ("mu", C.POINTER(C.c_float)), ("isd", C.POINTER(C.c_float)), ("tsc", C.c_double), ("X", C.c_void_p),
        ("T", C.c_void_p),
    ]


class TailPredictArgs(C.Structure):
    _fields_ = [
        ("chi_t", C.c_void_p), ("chi_h", C.c_void_p), ("qpg", _f64p), ("mill_g", C.POINTER(C.c_int32)),
        ("bvec", _f64p), ("w", _f64p), ("ng", C.c_int), ("nw", C.c_int), ("mu", C.POINTER(C.c_float)),
        ("isd", C.POINTER(C.c_float)), ("lo", C.POINTER(C.c_float)), ("hi", C.POINTER(C.c_float)),
        ("nl", C.c_int), ("dims", C.POINTER(C.c_int)), ("nmem", C.c_int), ("params", C.c_void_p),
        ("Y", C.c_void_p), ("stats", C.c_void_p),
    ]


class XtermArgs(C.Structure):
    _fields_ = [
        ("npw_v", C.c_int), ("mill_v", C.POINTER(C.c_int32)), ("nv", C.c_int), ("coef_v", C.c_void_p),
        ("e_v", C.c_void_p), ("ebar", C.c_double), ("ng", C.c_int), ("mill_g", C.POINTER(C.c_int32)),
        ("nw", C.c_int), ("w", _f64p), ("pref", C.c_double), ("nn", C.c_int), ("rho", C.c_void_p),
        ("out", C.c_void_p), ("prec", C.c_int),
    ]


class Chi0RealArgs(C.Structure):
    _fields_ = [("nt", C.c_int), ("ng", C.c_int), ("nw", C.c_int), ("prec", C.c_int), ("rho", C.c_void_p),
                ("dE", C.c_void_p), ("w", _f64p), ("eta", C.c_double), ("pref", C.c_double),
                ("accumulate", C.c_int), ("check_dE", C.c_int), ("chi0", C.c_void_p)]


class PpaArgs(C.Structure):
    _fields_ = [("ng", C.c_int), ("einv0", C.c_void_p), ("einvp", C.c_void_p), ("omega_p", C.c_double),
                ("qpg", _f64p), ("q0", C.c_int), ("nk_omega", C.c_double), ("wr", C.c_void_p), ("om", C.c_void_p)]


class SigmaArgs(C.Structure):
    _fields_ = [("nm", C.c_int), ("nn", C.c_int), ("ng", C.c_int), ("nz", C.c_int), ("rho", C.c_void_p),
                ("wr", C.c_void_p), ("om", C.c_void_p), ("e_m", C.c_void_p), ("f_m", C.c_void_p),
                ("z", C.c_void_p), ("eta", C.c_double), ("nk_omega", C.c_double), ("qpg", _f64p),
                ("q0", C.c_int), ("sigx", C.c_void_p), ("sigc", C.c_void_p), ("accumulate", C.c_int),
                ("rho_swapped", C.c_int)]


class Tune(C.Structure):
    _fields_ = [("nt_tiles", C.c_int), ("kper", C.c_int), ("wg_per_cu", C.c_int)]


class XoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRNAME.get(code, code)}: {msg}")
        self.code = code


_LIB = None

EXPORTS = ("xo_last_error", "xo_version", "xo_release_workspace", "xo_timing_enable", "xo_timing_report",
           "xo_rho", "xo_rho_batch", "xo_chi0", "xo_chi0_batch", "xo_chi0_autotune", "xo_epsinv", "xo_mlp_forward", "xo_mlp_backward", "xo_mse",
           "xo_adam_step", "xo_gather_rows", "xo_col_stats", "xo_tail_features", "xo_tail_apply", "xo_tail_guard",
           "xo_xterm", "xo_ppa_fit", "xo_sigma", "xo_chi0_real", "xo_rho_workspace_size",
           "xo_chi0_workspace_size", "xo_epsinv_workspace_size", "xo_epsinv_noalloc", "xo_tail_predict")


def lib():
    """Load libxo.so (raises if it was not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1902_03837_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.xo_last_error.restype = C.c_char_p
        L.xo_version.restype = C.c_char_p
        for name, argt in (("xo_rho", RhoArgs), ("xo_chi0", Chi0Args), ("xo_epsinv", EpsArgs),
                           ("xo_xterm", XtermArgs), ("xo_ppa_fit", PpaArgs), ("xo_sigma", SigmaArgs),
                           ("xo_chi0_real", Chi0RealArgs)):
            fn = getattr(L, name)
            fn.argtypes = [C.POINTER(argt), C.c_void_p]
            fn.restype = C.c_int
        vp, ip, i, l, f = C.c_void_p, C.POINTER(C.c_int), C.c_int, C.c_long, C.c_float
        fp = C.POINTER(C.c_float)
        L.xo_mlp_forward.argtypes = [i, ip, vp, vp, i, vp, vp, vp]
        L.xo_mlp_backward.argtypes = [i, ip, vp, vp, i, vp, vp, vp, vp, vp, vp]
        L.xo_mse.argtypes = [vp, vp, l, vp, vp, vp, vp]
        L.xo_adam_step.argtypes = [vp, vp, vp, vp, l, f, f, f, f, i, vp]
        L.xo_gather_rows.argtypes = [vp, vp, i, i, vp, vp]
        L.xo_col_stats.argtypes = [vp, l, i, vp, vp]
        L.xo_col_stats.restype = C.c_int
        L.xo_tail_features.argtypes = [C.POINTER(TailArgs), vp]
        L.xo_tail_predict.argtypes = [C.POINTER(TailPredictArgs), vp]
        L.xo_tail_apply.argtypes = [vp, vp, vp, _f64p, i, i, C.c_double, vp, vp]
        L.xo_tail_guard.argtypes = [vp, l, i, fp, fp, vp, vp, i, vp, vp]
        for nm in ("xo_mlp_forward", "xo_mlp_backward", "xo_mse", "xo_adam_step", "xo_gather_rows",
                   "xo_tail_features", "xo_tail_apply", "xo_tail_guard", "xo_tail_predict"):
            getattr(L, nm).restype = C.c_int
        L.xo_rho_batch.argtypes = [C.POINTER(RhoArgs), C.c_int, C.c_void_p]
        L.xo_chi0_batch.argtypes = [C.POINTER(Chi0Args), C.c_int, C.POINTER(Tune), C.c_void_p]
        L.xo_chi0_batch.restype = C.c_int
        L.xo_chi0_autotune.argtypes = [C.POINTER(Chi0Args), C.c_int, C.POINTER(Tune), C.POINTER(C.c_double),
                                       C.c_void_p]
        L.xo_chi0_autotune.restype = C.c_int
        L.xo_rho_batch.restype = C.c_int
        L.xo_release_workspace.restype = C.c_int
        L.xo_timing_enable.argtypes = [C.c_int]
        L.xo_timing_enable.restype = C.c_int
        L.xo_timing_report.argtypes = [C.c_char_p, C.c_int]
        L.xo_timing_report.restype = C.c_int
        _LIB = L
    return _LIB


def _check(rc: int):
    if rc != XO_OK:
        raise XoError(rc, lib().xo_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _host_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(t) -> int:
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return t.data_ptr()


def version() -> str:
    return lib().xo_version().decode()


def release_workspace():
    _check(lib().xo_release_workspace())


def timing_enable(on: bool = True):
    _check(lib().xo_timing_enable(1 if on else 0))


def timing_report() -> dict:
    """{kernel: (launches, total_ms)} since the last report (synchronises)."""
    buf = C.create_string_buffer(1 << 16)
    _check(lib().xo_timing_report(buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms = line.split()
        out[name] = (int(n), float(ms))
    return out


def _cdtype(prec):
    import torch
    return torch.complex128 if (PREC[prec] if isinstance(prec, str) else int(prec)) == XO_FP64 else torch.complex64


def _rho_args(coef_c, mill_c, e_c, coef_v, mill_v, e_v, gmill, g0, grid, *, out, dE=None,
              prec="fp64", kcart=(0., 0., 0.), bvec=None, q0=False, qhat=(1., 0., 0.)):
    """Checked argument block for one k-pair (returns it with the host arrays it points to)."""
    import torch
    mc, mv, mg = _host_i32(mill_c), _host_i32(mill_v), _host_i32(gmill)
    cdt = _cdtype(prec)
    nc, nv, ng = coef_c.shape[0], coef_v.shape[0], mg.shape[0]
    # host-side shape checks: the kernels trust these extents
    assert mc.ndim == 2 and mc.shape[1] == 3 and mv.ndim == 2 and mv.shape[1] == 3 and mg.shape[1] == 3
    assert tuple(coef_c.shape) == (nc, mc.shape[0]) and coef_c.dtype == cdt, (coef_c.shape, coef_c.dtype)
    assert tuple(coef_v.shape) == (nv, mv.shape[0]) and coef_v.dtype == cdt, (coef_v.shape, coef_v.dtype)
    assert tuple(out.shape) == (nv, nc, ng) and out.dtype == cdt, (out.shape, out.dtype)
    if dE is not None:
        assert dE.numel() == nv * nc and dE.dtype == torch.float64
    if dE is not None or q0:
        assert e_c is not None and e_v is not None
        assert e_c.numel() >= nc and e_v.numel() >= nv and e_c.dtype == e_v.dtype == torch.float64
    a = RhoArgs()
    a.n[:] = [int(x) for x in grid]
    a.bvec[:] = list(np.asarray(bvec if bvec is not None else np.eye(3), float).reshape(9))
    a.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    a.npw_c, a.mill_c, a.nc = mc.shape[0], mc.ctypes.data_as(_i32p), coef_c.shape[0]
    a.coef_c, a.e_c = _ptr(coef_c), _ptr(e_c)
    a.kcart[:] = [float(x) for x in kcart]
    a.npw_v, a.mill_v, a.nv = mv.shape[0], mv.ctypes.data_as(_i32p), coef_v.shape[0]
    a.coef_v, a.e_v = _ptr(coef_v), _ptr(e_v)
    a.g0[:] = [int(x) for x in g0]
    a.ng, a.mill_g = mg.shape[0], mg.ctypes.data_as(_i32p)
    a.q0 = 1 if q0 else 0
    a.qhat[:] = [float(x) for x in qhat]
    a.rho, a.dE = _ptr(out), _ptr(dE)
    return a, (mc, mv, mg)


def rho(coef_c, mill_c, e_c, coef_v, mill_v, e_v, gmill, g0, grid, *, out, dE=None,
        prec="fp64", kcart=(0., 0., 0.), bvec=None, q0=False, qhat=(1., 0., 0.), stream=None):
    """xo_rho for one k-pair: out[nv][nc][ng] (and dE[nv][nc] if given)."""
    a, keep = _rho_args(coef_c, mill_c, e_c, coef_v, mill_v, e_v, gmill, g0, grid, out=out, dE=dE,
                        prec=prec, kcart=kcart, bvec=bvec, q0=q0, qhat=qhat)
    _check(lib().xo_rho(C.byref(a), _stream(stream)))
    return out


class RhoPlan:
    """Checked argument blocks for a fixed set of pairs and buffers, reusable across calls."""

    def __init__(self, pairs, batch=True, ntrans=0):
        self.built = [_rho_args(**kw) for kw in pairs]
        self.arr = (RhoArgs * len(self.built))(*[b[0] for b in self.built])
        self.batch = batch
        self.ntrans = ntrans


def launch_plan(plan: RhoPlan, stream=None):
    st = _stream(stream)
    if plan.batch:
        _check(lib().xo_rho_batch(plan.arr, len(plan.built), st))
    else:
        for i in range(len(plan.built)):
            _check(lib().xo_rho(C.byref(plan.arr[i]), st))


def rho_workspace_size(arr, n=None):
    """xo_rho_workspace_size over a RhoPlan or a ctypes array of RhoArgs: device bytes."""
    if isinstance(arr, RhoPlan):
        arr, n = arr.arr, len(arr.built)
    out = C.c_size_t(0)
    _check(lib().xo_rho_workspace_size(arr, int(n if n is not None else len(arr)), C.byref(out)))
    return out.value


def chi0_workspace_size(items, tune=None):
    """xo_chi0_workspace_size over a list of Chi0Args (and an optional Tune): device bytes."""
    arr = (Chi0Args * len(items))(*items)
    out = C.c_size_t(0)
    _check(lib().xo_chi0_workspace_size(arr, len(items), C.byref(tune) if tune is not None else None,
                                        C.byref(out)))
    return out.value


def epsinv_workspace_size(ng, nw):
    """xo_epsinv_workspace_size for ng G-vectors and nw frequencies: device bytes."""
    a = EpsArgs()
    a.ng, a.nw = int(ng), int(nw)
    out = C.c_size_t(0)
    _check(lib().xo_epsinv_workspace_size(C.byref(a), C.byref(out)))
    return out.value


def rho_batch(pairs, stream=None):
    """xo_rho_batch over a list of keyword dicts, each as for rho()."""
    built = [_rho_args(**kw) for kw in pairs]
    arr = (RhoArgs * len(built))(*[b[0] for b in built])
    _check(lib().xo_rho_batch(arr, len(built), _stream(stream)))


def chi0(rho_m, dE, omegas: Sequence[float], pref: float, *, out, prec="fp64", accumulate=False,
         check_dE=True, stream=None):
    """xo_chi0: out[nw][ng][ng] complex128 (+)= -pref sum_t W_t(w) rho_t rho_t^H."""
    import torch
    w = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
    assert rho_m.ndim == 2 and rho_m.dtype == _cdtype(prec), (rho_m.shape, rho_m.dtype)
    assert dE.numel() == rho_m.shape[0] and dE.dtype == torch.float64
    assert tuple(out.shape) == (w.shape[0], rho_m.shape[1], rho_m.shape[1]) and out.dtype == torch.complex128
    a = Chi0Args()
    a.nt, a.ng, a.nw = rho_m.shape[0], rho_m.shape[1], w.shape[0]
    a.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    a.rho, a.dE, a.w, a.pref = _ptr(rho_m), _ptr(dE), w.ctypes.data_as(_f64p), float(pref)
    a.accumulate, a.check_dE, a.chi0 = int(bool(accumulate)), int(bool(check_dE)), _ptr(out)
    _check(lib().xo_chi0(C.byref(a), _stream(stream)))
    return out


def _chi0_args(rho_m, dE, omegas, pref, out, prec, accumulate, check_dE):
    import torch
    w = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
    assert rho_m.ndim == 2 and rho_m.dtype == _cdtype(prec), (rho_m.shape, rho_m.dtype)
    assert dE.numel() == rho_m.shape[0] and dE.dtype == torch.float64
    assert tuple(out.shape) == (w.shape[0], rho_m.shape[1], rho_m.shape[1]) and out.dtype == torch.complex128
    a = Chi0Args()
    a.nt, a.ng, a.nw = rho_m.shape[0], rho_m.shape[1], w.shape[0]
    a.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    a.rho, a.dE, a.w, a.pref = _ptr(rho_m), _ptr(dE), w.ctypes.data_as(_f64p), float(pref)
    a.accumulate, a.check_dE, a.chi0 = int(bool(accumulate)), int(bool(check_dE)), _ptr(out)
    return a, w


def chi0_batch(items, omegas, *, prec="fp64", tune=None, check_dE=True, stream=None):
    """xo_chi0_batch over items = [(rho, dE, pref, out), ...] sharing the frequencies."""
    built = [_chi0_args(r, d, omegas, p, o, prec, False, check_dE) for r, d, p, o in items]
    arr = (Chi0Args * len(built))(*[b[0] for b in built])
    t = None
    if tune is not None:
        t = Tune(*[int(x) for x in tune])
    _check(lib().xo_chi0_batch(arr, len(built), C.byref(t) if t is not None else None, _stream(stream)))


def chi0_autotune(items, omegas, *, prec="fp64", stream=None):
    """Fastest (nt_tiles, kper, wg_per_cu) for this batch and its time in ms."""
    built = [_chi0_args(r, d, omegas, p, o, prec, False, False) for r, d, p, o in items]
    arr = (Chi0Args * len(built))(*[b[0] for b in built])
    t = Tune()
    ms = C.c_double()
    _check(lib().xo_chi0_autotune(arr, len(built), C.byref(t), C.byref(ms), _stream(stream)))
    return (t.nt_tiles, t.kper, t.wg_per_cu), ms.value


def epsinv(chi0_m, qpg, *, out, flags=XO_EPS_SYM, info=None, stream=None, noalloc=False):
    """xo_epsinv: out = eps~^-1 (or (I - v chi0)^-1 with XO_EPS_NONSYM), complex128.

    info: optional int32 device tensor [nw]; when given the call does not synchronise and
    the pivot flags land there (0: frequency passed, else 1 + its first failing pivot).
    noalloc: call xo_epsinv_noalloc (static scratch, no allocation) instead."""
    import torch
    q = np.ascontiguousarray(np.asarray(qpg, dtype=np.float64))
    assert chi0_m.ndim == 3 and chi0_m.shape[1] == chi0_m.shape[2] == q.shape[0]
    assert chi0_m.dtype == torch.complex128 and out.dtype == torch.complex128
    assert tuple(out.shape) == tuple(chi0_m.shape)
    a = EpsArgs()
    a.ng, a.nw = chi0_m.shape[-1], chi0_m.shape[0]
    a.qpg, a.chi0, a.flags, a.out = q.ctypes.data_as(_f64p), _ptr(chi0_m), int(flags), _ptr(out)
    if info is not None:
        assert info.dtype == torch.int32 and info.numel() == a.nw and info.is_contiguous()
        a.info = _ptr(info)
    fn = lib().xo_epsinv_noalloc if noalloc else lib().xo_epsinv
    _check(fn(C.byref(a), _stream(stream)))
    return out


# --------------------------------------------------------------------------- MLP / tail

def _dims(dims):
    d = (C.c_int * len(dims))(*[int(x) for x in dims])
    return d


def mlp_forward(dims, params, X, n, acts, Y, stream=None):
    _check(lib().xo_mlp_forward(len(dims) - 1, _dims(dims), _ptr(params), _ptr(X), int(n), _ptr(acts), _ptr(Y),
                                _stream(stream)))


def mlp_backward(dims, params, X, n, acts, dY, grads, work, dX=None, stream=None):
    _check(lib().xo_mlp_backward(len(dims) - 1, _dims(dims), _ptr(params), _ptr(X), int(n), _ptr(acts), _ptr(dY),
                                 _ptr(grads), _ptr(work), _ptr(dX), _stream(stream)))


def mse(Y, T, dY, loss, partial, stream=None):
    assert Y.numel() == T.numel() and (dY is None or dY.numel() == Y.numel()) and partial.numel() >= 256
    _check(lib().xo_mse(_ptr(Y), _ptr(T), Y.numel(), _ptr(dY), _ptr(loss), _ptr(partial), _stream(stream)))


def adam_step(p, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    assert p.numel() == g.numel() == m.numel() == v.numel()
    _check(lib().xo_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), lr, b1, b2, eps, int(step),
                              _stream(stream)))


def gather_rows(src, idx, dst, stream=None):
    n, F = dst.shape
    assert src.shape[1] == F and idx.numel() == n and idx.dtype.itemsize == 4
    _check(lib().xo_gather_rows(_ptr(src), _ptr(idx), n, F, _ptr(dst), _stream(stream)))


def _geo(qpg, mill_g, bvec, w, ng, nw):
    q = np.ascontiguousarray(np.asarray(qpg, np.float64))
    m = np.ascontiguousarray(np.asarray(mill_g, np.int32))
    b = np.ascontiguousarray(np.asarray(bvec, np.float64))
    ww = np.ascontiguousarray(np.asarray(w, np.float64))
    assert q.size == ng and m.shape == (ng, 3) and b.shape == (3, 3) and ww.size == nw
    return q, m, b, ww


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float32))


def tail_features(chi_t, chi_h, qpg, mill_g, bvec, w, mu, isd, X, chi_f=None, T=None, tsc=1.0, stream=None):
    nw, ng = chi_t.shape[0], chi_t.shape[1]
    assert X.shape == (nw * ng * ng, 9) and chi_h.shape == chi_t.shape
    if T is not None:
        assert chi_f is not None and T.shape == (nw * ng * ng, 2)
    q, m, b, ww = _geo(qpg, mill_g, bvec, w, ng, nw)
    keepf = [_f32(mu), _f32(isd)]
    a = TailArgs()
    a.chi_t, a.chi_h, a.chi_f = _ptr(chi_t), _ptr(chi_h), _ptr(chi_f)
    a.qpg, a.bvec, a.w = (k.ctypes.data_as(_f64p) for k in (q, b, ww))
    a.mill_g = m.ctypes.data_as(C.POINTER(C.c_int32))
    a.ng, a.nw = ng, nw
    a.mu, a.isd = (k.ctypes.data_as(C.POINTER(C.c_float)) for k in keepf)
    a.tsc, a.X, a.T = float(tsc), _ptr(X), _ptr(T)
    _check(lib().xo_tail_features(C.byref(a), _stream(stream)))


def tail_predict(chi_t, chi_h, qpg, mill_g, bvec, w, mu, isd, lo, hi, dims, params, Y, stats, stream=None):
    """xo_tail_predict: Y [n][2] = ensemble mean of the tail MLPs (bf16 matrix cores) on the
    features of every element, stats [3] = guard sums. params: FP32 device tensor [nmem][P]."""
    import torch
    nw, ng = chi_t.shape[0], chi_t.shape[1]
    assert chi_h.shape == chi_t.shape and Y.shape == (nw * ng * ng, 2) and stats.numel() >= 3
    assert params.dim() == 2 and params.is_contiguous() and params.dtype == torch.float32
    assert params.shape[1] == sum(a * b + b for a, b in zip(dims[:-1], dims[1:])), "params do not match dims"
    q, m, b, ww = _geo(qpg, mill_g, bvec, w, ng, nw)
    keepf = [_f32(mu), _f32(isd), _f32(lo), _f32(hi)]
    d = np.ascontiguousarray(np.asarray(dims, np.int32))
    a = TailPredictArgs()
    a.chi_t, a.chi_h = _ptr(chi_t), _ptr(chi_h)
    a.qpg, a.bvec, a.w = (k.ctypes.data_as(_f64p) for k in (q, b, ww))
    a.mill_g = m.ctypes.data_as(C.POINTER(C.c_int32))
    a.ng, a.nw = ng, nw
    a.mu, a.isd, a.lo, a.hi = (k.ctypes.data_as(C.POINTER(C.c_float)) for k in keepf)
    a.nl, a.dims = len(d) - 1, d.ctypes.data_as(C.POINTER(C.c_int))
    a.nmem, a.params = params.shape[0], _ptr(params)
    a.Y, a.stats = _ptr(Y), _ptr(stats)
    _check(lib().xo_tail_predict(C.byref(a), _stream(stream)))


def tail_apply(chi_t, Y1, qpg, tsc, out, Y2=None, stream=None):
    nw, ng = chi_t.shape[0], chi_t.shape[1]
    q = np.ascontiguousarray(np.asarray(qpg, np.float64))
    assert Y1.numel() == nw * ng * ng * 2 and out.shape == chi_t.shape
    assert Y2 is None or Y2.numel() == Y1.numel()
    _check(lib().xo_tail_apply(_ptr(chi_t), _ptr(Y1), _ptr(Y2), q.ctypes.data_as(_f64p), ng, nw, float(tsc),
                               _ptr(out), _stream(stream)))


def tail_guard(X, lo, hi, Y1, Y2, stats, stream=None):
    n, F = X.shape
    lo_ = np.ascontiguousarray(np.asarray(lo, np.float32))
    hi_ = np.ascontiguousarray(np.asarray(hi, np.float32))
    ny = Y1.shape[1]
    assert Y2.shape == Y1.shape and Y1.shape[0] == n and stats.numel() >= 3
    _check(lib().xo_tail_guard(_ptr(X), n, F, lo_.ctypes.data_as(C.POINTER(C.c_float)),
                               hi_.ctypes.data_as(C.POINTER(C.c_float)), _ptr(Y1), _ptr(Y2), ny, _ptr(stats),
                               _stream(stream)))


def col_stats(X, out, stream=None):
    n, F = X.shape
    assert out.numel() >= 4 * F
    _check(lib().xo_col_stats(_ptr(X), n, F, _ptr(out), _stream(stream)))


def xterm(coef_v, mill_v, e_v, ebar, gmill, omegas, pref, rho_m, nn, out, prec="fp64", stream=None):
    """xo_xterm: out[nw][ng][ng] (complex128) += Bruneval-Gonze correction of one k-pair.

    coef_v [nv][npw_v] and e_v [nv] float64 on the device; rho_m [nv*nn][ng] from xo_rho
    over the nn explicit bands at k; coef_v and rho_m are complex128 for "fp64", complex64
    for the other precisions (the explicit-band update then runs in that precision)."""
    import torch
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    assert coef_v.dtype == cdt and e_v.dtype == torch.float64 and rho_m.dtype == cdt
    nv, npw = coef_v.shape
    mv = _host_i32(mill_v)
    mg = _host_i32(gmill)
    w = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
    assert mv.shape == (npw, 3) and e_v.numel() == nv and tuple(rho_m.shape) == (nv * nn, mg.shape[0])
    assert tuple(out.shape) == (w.shape[0], mg.shape[0], mg.shape[0]) and out.dtype == torch.complex128
    a = XtermArgs()
    a.npw_v, a.mill_v, a.nv = npw, mv.ctypes.data_as(C.POINTER(C.c_int32)), nv
    a.coef_v, a.e_v, a.ebar = _ptr(coef_v), _ptr(e_v), float(ebar)
    a.ng, a.mill_g, a.nw, a.w = mg.shape[0], mg.ctypes.data_as(C.POINTER(C.c_int32)), w.shape[0], w.ctypes.data_as(_f64p)
    a.pref, a.nn, a.rho, a.out = float(pref), int(nn), _ptr(rho_m), _ptr(out)
    a.prec = PREC[prec]
    _check(lib().xo_xterm(C.byref(a), _stream(stream)))
    return out


def _host_f64(a, n):
    v = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    assert v.shape == (n,), (v.shape, n)
    return v


def ppa_fit(einv0, einvp, omega_p, qpg, *, q0=False, nk_omega=0.0, wr, om, stream=None):
    """xo_ppa_fit: plasmon-pole residue of W_c (wr) and pole energies (om), [ng][ng] complex128.
    qpg: |q+G| per G (host); q0: q = 0 with G = 0 first (then nk_omega = N_k Omega is used)."""
    import torch
    ng = einv0.shape[-1]
    for t in (einv0, einvp, wr, om):
        assert tuple(t.shape) == (ng, ng) and t.dtype == torch.complex128 and t.is_contiguous()
    qg = _host_f64(qpg, ng)
    a = PpaArgs()
    a.ng, a.einv0, a.einvp, a.omega_p = ng, _ptr(einv0), _ptr(einvp), float(omega_p)
    a.qpg, a.q0, a.nk_omega = qg.ctypes.data_as(_f64p), 1 if q0 else 0, float(nk_omega)
    a.wr, a.om = _ptr(wr), _ptr(om)
    _check(lib().xo_ppa_fit(C.byref(a), _stream(stream)))
    return wr, om


def sigma(rho_m, wr, om, e_m, f_m, z, eta, nk_omega, *, sigc=None, sigx=None, qpg=None, q0=False,
          accumulate=False, swapped=False, stream=None):
    """xo_sigma for one q: sigc[nn][nz] (complex128) and sigx[nn] (float64), (+)=.

    rho_m [nm][nn][ng] complex128 (xo_rho with the states n on the conduction side), or with
    swapped=True [nn][nm][ng] from xo_rho with the bands on the conduction side, G0 and the
    G-set negated; e_m, f_m [nm] float64 and z [nn][nz] complex128 on the device; nk_omega =
    N_k Omega (the prefactor is its inverse); qpg (host, |q+G|) is needed for Sigma_x."""
    import torch
    if swapped:
        nn, nm, ng = rho_m.shape
    else:
        nm, nn, ng = rho_m.shape
    assert rho_m.dtype == torch.complex128 and rho_m.is_contiguous()
    assert e_m.dtype == f_m.dtype == torch.float64 and e_m.numel() == nm and f_m.numel() == nm
    nz = 0 if z is None else z.shape[1]
    if nz:
        assert tuple(z.shape) == (nn, nz) and z.dtype == torch.complex128 and z.is_contiguous()
        assert sigc is not None and tuple(sigc.shape) == (nn, nz) and sigc.dtype == torch.complex128
        for t in (wr, om):
            assert tuple(t.shape) == (ng, ng) and t.dtype == torch.complex128 and t.is_contiguous()
    if sigx is not None:
        assert tuple(sigx.shape) == (nn,) and sigx.dtype == torch.float64 and qpg is not None
    qg = _host_f64(qpg, ng) if qpg is not None else None
    a = SigmaArgs()
    a.nm, a.nn, a.ng, a.nz = nm, nn, ng, nz
    a.rho, a.wr, a.om = _ptr(rho_m), _ptr(wr) if nz else None, _ptr(om) if nz else None
    a.e_m, a.f_m, a.z = _ptr(e_m), _ptr(f_m), _ptr(z) if nz else None
    a.eta, a.nk_omega = float(eta), float(nk_omega)
    a.qpg = qg.ctypes.data_as(_f64p) if qg is not None else None
    a.q0 = 1 if q0 else 0
    a.sigx = _ptr(sigx) if sigx is not None else None
    a.sigc = _ptr(sigc) if nz else None
    a.accumulate = 1 if accumulate else 0
    a.rho_swapped = 1 if swapped else 0
    _check(lib().xo_sigma(C.byref(a), _stream(stream)))
    return sigc, sigx


def chi0_real(rho_m, dE, omegas, eta, pref, *, out, prec="fp64", accumulate=False, check_dE=True, stream=None):
    """xo_chi0_real: out[nw][ng][ng] complex128 (+)= pref sum_t F_t(w) rho_t rho_t^H at real w."""
    import torch
    nt, ng = rho_m.shape
    assert rho_m.dtype == _cdtype(prec) and rho_m.is_contiguous()
    assert dE.dtype == torch.float64 and dE.numel() == nt
    w = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64).reshape(-1))
    assert tuple(out.shape) == (w.shape[0], ng, ng) and out.dtype == torch.complex128 and out.is_contiguous()
    a = Chi0RealArgs()
    a.nt, a.ng, a.nw = nt, ng, w.shape[0]
    a.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    a.rho, a.dE, a.w = _ptr(rho_m), _ptr(dE), w.ctypes.data_as(_f64p)
    a.eta, a.pref = float(eta), float(pref)
    a.accumulate, a.check_dE, a.chi0 = 1 if accumulate else 0, 1 if check_dE else 0, _ptr(out)
    _check(lib().xo_chi0_real(C.byref(a), _stream(stream)))
    return out

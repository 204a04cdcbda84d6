"""C-ABI library: loads, exports every declared symbol, validates arguments on the host.

CPU only: no call here reaches a kernel launch (each fails validation first).
"""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1902_03837_amd import xo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "xo.h")).read()
    return sorted(set(re.findall(r"\b(xo_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = xo.lib()
    names = _declared()
    assert {"xo_rho", "xo_chi0", "xo_epsinv", "xo_last_error", "xo_version"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert set(xo.EXPORTS) <= set(names)
    assert xo.version().startswith("xo ")


def test_struct_layouts_match_header_sizes():
    # field counts of the ctypes mirrors track the header structs
    src = open(os.path.join(ROOT, "include", "xo.h")).read()
    assert "xo_rho_args" in src and "xo_chi0_args" in src and "xo_eps_args" in src
    assert C.sizeof(xo.Chi0Args) == 4 * 4 + 3 * 8 + 8 + 4 + 4 + 8
    assert C.sizeof(xo.EpsArgs) == 8 + 8 + 8 + 8 + 8 + 8


def _rc(fn, a):
    rc = fn(C.byref(a), None)
    return rc, xo.lib().xo_last_error().decode()


def test_chi0_argument_errors():
    L = xo.lib()
    a = xo.Chi0Args()
    rc, msg = _rc(L.xo_chi0, a)
    assert rc == xo.XO_ERR_ARG and "positive" in msg
    w = np.array([0.0, -1.0])
    a.nt, a.ng, a.nw, a.prec = 4, 3, 2, 0
    a.rho, a.dE, a.chi0 = 8, 8, 8   # never dereferenced: validation fails first
    a.w = w.ctypes.data_as(C.POINTER(C.c_double))
    a.pref = 1.0
    rc, msg = _rc(L.xo_chi0, a)
    assert rc == xo.XO_ERR_ARG and "negative" in msg
    w[1] = 1.0
    a.prec = 7
    rc, msg = _rc(L.xo_chi0, a)
    assert rc == xo.XO_ERR_ARG and "precision" in msg
    a.prec = 0
    a.nw = 65
    rc, msg = _rc(L.xo_chi0, a)
    assert rc == xo.XO_ERR_ARG


def _rho_args(mc, mv, mg, grid, g0=(0, 0, 0)):
    a = xo.RhoArgs()
    a.n[:] = grid
    keep = [np.ascontiguousarray(x, dtype=np.int32) for x in (mc, mv, mg)]
    a.npw_c, a.mill_c = len(mc), keep[0].ctypes.data_as(C.POINTER(C.c_int32))
    a.npw_v, a.mill_v = len(mv), keep[1].ctypes.data_as(C.POINTER(C.c_int32))
    a.ng, a.mill_g = len(mg), keep[2].ctypes.data_as(C.POINTER(C.c_int32))
    a.nc = a.nv = 2
    a.coef_c = a.coef_v = a.rho = 8
    a.g0[:] = g0
    return a, keep


def test_rho_alias_and_wrap_checks():
    L = xo.lib()
    sphere = np.array([[i, j, k] for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4)])
    gs = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0]])
    # reach along x: 3 - (-3) - (-1) = 7 -> needs N >= 8; the sphere spans 7 -> N >= 7
    a, keep = _rho_args(sphere, sphere, gs, [7, 16, 16])
    rc, msg = _rc(L.xo_rho, a)
    assert rc == xo.XO_ERR_ARG and "aliases" in msg
    a, keep = _rho_args(sphere, sphere, gs, [6, 16, 16])
    rc, msg = _rc(L.xo_rho, a)
    assert rc == xo.XO_ERR_ARG and "wraps" in msg
    a, keep = _rho_args(sphere, sphere, gs, [200, 16, 16])
    rc, msg = _rc(L.xo_rho, a)
    assert rc == xo.XO_ERR_UNSUPPORTED
    # q0 needs G = 0 in the G-set
    a, keep = _rho_args(sphere, sphere, gs[1:], [16, 16, 16])
    a.q0 = 1
    a.qhat[:] = [1, 0, 0]
    a.e_c = a.e_v = 8
    rc, msg = _rc(L.xo_rho, a)
    assert rc == xo.XO_ERR_ARG and "G = 0" in msg


def test_epsinv_argument_errors():
    L = xo.lib()
    q = np.array([1.0, 0.0, 2.0])
    a = xo.EpsArgs()
    a.ng, a.nw = 3, 1
    a.qpg = q.ctypes.data_as(C.POINTER(C.c_double))
    a.chi0, a.out = 8, 16
    rc, msg = _rc(L.xo_epsinv, a)
    assert rc == xo.XO_ERR_ARG and "|q+G|" in msg
    a.flags = 64
    rc, msg = _rc(L.xo_epsinv, a)
    assert rc == xo.XO_ERR_ARG and "flags" in msg


def test_xterm_argument_errors():
    L = xo.lib()
    a = xo.XtermArgs()
    rc, msg = _rc(L.xo_xterm, a)
    assert rc == xo.XO_ERR_ARG and "positive" in msg
    mv = np.zeros((2, 3), dtype=np.int32)
    mv[1, 0] = 1
    mg = np.zeros((1, 3), dtype=np.int32)
    w = np.array([0.0, -0.5])
    a.npw_v, a.nv, a.ng, a.nw, a.nn = 2, 1, 1, 2, 1
    a.mill_v = mv.ctypes.data_as(C.POINTER(C.c_int32))
    a.mill_g = mg.ctypes.data_as(C.POINTER(C.c_int32))
    a.w = w.ctypes.data_as(C.POINTER(C.c_double))
    rc, msg = _rc(L.xo_xterm, a)
    assert rc == xo.XO_ERR_ARG and "null device pointer" in msg
    a.coef_v = a.e_v = a.rho = a.out = 8   # never dereferenced: validation fails first
    a.pref, a.ebar = 1.0, 2.0
    rc, msg = _rc(L.xo_xterm, a)
    assert rc == xo.XO_ERR_ARG and "negative" in msg
    w[1] = 0.5
    mv[1, 0] = 0   # a repeated Miller vector
    rc, msg = _rc(L.xo_xterm, a)
    assert rc == xo.XO_ERR_ARG and "repeats" in msg


def test_empty_and_degenerate_inputs_are_rejected():
    """Zero bands, zero G vectors, empty batches and zero-row MLP batches fail validation
    with XO_ERR_ARG before any device work."""
    L = xo.lib()
    sphere = np.array([[i, j, k] for i in range(-1, 2) for j in range(-1, 2) for k in range(-1, 2)])
    gs = np.array([[0, 0, 0], [1, 0, 0]])
    for field in ("nc", "nv"):
        a, keep = _rho_args(sphere, sphere, gs, [8, 8, 8])
        setattr(a, field, 0)
        rc, msg = _rc(L.xo_rho, a)
        assert rc == xo.XO_ERR_ARG and "positive" in msg, (field, msg)
    a, keep = _rho_args(sphere, sphere, gs[:0], [8, 8, 8])
    rc, msg = _rc(L.xo_rho, a)
    assert rc == xo.XO_ERR_ARG
    assert L.xo_rho_batch(None, 0, None) == xo.XO_ERR_ARG
    assert L.xo_chi0_batch(None, 0, None, None) == xo.XO_ERR_ARG
    best, ms = xo.Tune(), C.c_double()
    assert L.xo_chi0_autotune(None, 0, C.byref(best), C.byref(ms), None) == xo.XO_ERR_ARG
    e = xo.EpsArgs()
    rc, msg = _rc(L.xo_epsinv, e)
    assert rc == xo.XO_ERR_ARG and "positive" in msg
    q = np.ones(2)
    e.ng, e.nw, e.qpg, e.chi0, e.out = 2, 1, q.ctypes.data_as(C.POINTER(C.c_double)), 8, 8
    rc, msg = _rc(L.xo_epsinv, e)
    assert rc == xo.XO_ERR_ARG and "alias" in msg
    dims = (C.c_int * 2)(4, 4)
    assert L.xo_mlp_forward(1, dims, 8, 8, 0, 8, 8, None) == xo.XO_ERR_ARG
    assert L.xo_mse(8, 8, 0, 8, 8, 8, None) == xo.XO_ERR_ARG
    assert L.xo_gather_rows(8, 8, 0, 4, 8, None) == xo.XO_ERR_ARG


def test_ppa_and_sigma_argument_errors():
    L = xo.lib()
    assert C.sizeof(xo.PpaArgs) == 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert C.sizeof(xo.SigmaArgs) == 4 * 4 + 6 * 8 + 8 + 8 + 8 + 8 + 8 + 8 + 4 + 4
    a = xo.PpaArgs()
    rc, msg = _rc(L.xo_ppa_fit, a)
    assert rc == xo.XO_ERR_ARG and "positive" in msg
    qg = np.array([1.0, -2.0])
    a.ng, a.einv0, a.einvp, a.wr, a.om = 2, 8, 8, 8, 8   # never dereferenced
    a.omega_p = 0.0
    rc, msg = _rc(L.xo_ppa_fit, a)
    assert rc == xo.XO_ERR_ARG and "omega_p" in msg
    a.omega_p = 1.0
    rc, msg = _rc(L.xo_ppa_fit, a)
    assert rc == xo.XO_ERR_ARG and "null qpg" in msg
    a.qpg = qg.ctypes.data_as(C.POINTER(C.c_double))
    rc, msg = _rc(L.xo_ppa_fit, a)
    assert rc == xo.XO_ERR_ARG and "|q+G| at 1" in msg
    # at q = 0 the G = 0 entry is not read, but N_k Omega must be given
    qg0 = np.array([-5.0, 2.0])
    a.qpg, a.q0 = qg0.ctypes.data_as(C.POINTER(C.c_double)), 1
    rc, msg = _rc(L.xo_ppa_fit, a)
    assert rc == xo.XO_ERR_ARG and "nk_omega" in msg
    s = xo.SigmaArgs()
    rc, msg = _rc(L.xo_sigma, s)
    assert rc == xo.XO_ERR_ARG and "positive" in msg
    s.nm, s.nn, s.ng, s.nz = 3, 2, 2, 5
    s.rho = s.e_m = s.f_m = s.wr = s.om = s.z = s.sigc = 8
    rc, msg = _rc(L.xo_sigma, s)
    assert rc == xo.XO_ERR_ARG and "at most 4" in msg
    s.nz = 2
    rc, msg = _rc(L.xo_sigma, s)
    assert rc == xo.XO_ERR_ARG and "nk_omega" in msg
    s.nk_omega, s.eta = 100.0, -0.1
    rc, msg = _rc(L.xo_sigma, s)
    assert rc == xo.XO_ERR_ARG and "eta" in msg
    s.eta, s.sigx = 0.0, 8
    rc, msg = _rc(L.xo_sigma, s)
    assert rc == xo.XO_ERR_ARG and "qpg" in msg


def test_chi0_real_argument_errors():
    L = xo.lib()
    assert C.sizeof(xo.Chi0RealArgs) == 4 * 4 + 3 * 8 + 2 * 8 + 4 + 4 + 8
    a = xo.Chi0RealArgs()
    rc, msg = _rc(L.xo_chi0_real, a)
    assert rc == xo.XO_ERR_ARG and "positive" in msg
    w = np.array([0.5, -1.0])
    a.nt, a.ng, a.nw, a.prec = 4, 3, 2, 0
    a.rho, a.dE, a.chi0 = 8, 8, 8   # never dereferenced: validation fails first
    a.w = w.ctypes.data_as(C.POINTER(C.c_double))
    a.pref = 1.0
    rc, msg = _rc(L.xo_chi0_real, a)
    assert rc == xo.XO_ERR_ARG and "eta" in msg
    a.eta = 0.01
    rc, msg = _rc(L.xo_chi0_real, a)
    assert rc == xo.XO_ERR_ARG and "frequency 1" in msg


def _rho_block(cr, ip, prec, mills):
    """Argument block of pair ip with fake device pointers (the size query reads none)."""
    ik, ikp, g0 = cr.pairs[ip]
    nv, nc = cr.nocc_at(ikp), cr.coef[ik].shape[0] - cr.nocc_at(ik)
    a = xo.RhoArgs()
    a.n[:] = list(cr.grid)
    a.prec = xo.PREC[prec]
    mc = np.ascontiguousarray(cr.mill[ik], dtype=np.int32)
    mv = np.ascontiguousarray(cr.mill[ikp], dtype=np.int32)
    mg = np.ascontiguousarray(cr.gmill, dtype=np.int32)
    mills += [mc, mv, mg]
    a.npw_c, a.mill_c, a.nc, a.coef_c, a.e_c = mc.shape[0], mc.ctypes.data_as(C.POINTER(C.c_int32)), nc, 4096, 4096
    a.npw_v, a.mill_v, a.nv, a.coef_v, a.e_v = mv.shape[0], mv.ctypes.data_as(C.POINTER(C.c_int32)), nv, 8192, 8192
    a.g0[:] = [int(x) for x in g0]
    a.ng, a.mill_g = mg.shape[0], mg.ctypes.data_as(C.POINTER(C.c_int32))
    a.rho = 16384
    return a, nc, nv


def test_workspace_size_queries():
    """Host-only size queries: consistent with what the calls allocate and with each other."""
    from synth import crystal_for
    cr = crystal_for("c1_small")
    mills = []
    sizes = {}
    for prec in ("fp64", "fp32", "bf16x3", "bf16"):
        blocks = [_rho_block(cr, ip, prec, mills) for ip in range(len(cr.pairs))]
        arr = (xo.RhoArgs * len(blocks))(*[b[0] for b in blocks])
        sizes[prec] = xo.rho_workspace_size(arr, len(blocks))
        # one pair alone takes no more than the batch
        assert xo.rho_workspace_size(arr, 1) <= sizes[prec]
    # FP64 / FP32 read the coefficients in place; the bf16 forms convert every distinct band
    # set once (hi + lo words for bf16x3, one word for bf16): 8 and 4 bytes per entry
    assert sizes["fp64"] == 0 and sizes["fp32"] == 0
    assert sizes["bf16x3"] == 2 * sizes["bf16"] > 0
    ent = 0
    seen = set()
    for ik, ikp, _ in cr.pairs:
        for k, nb in ((ik, cr.coef[ik].shape[0] - cr.nocc_at(ik)), (ikp, cr.nocc_at(ikp))):
            if (k, nb) not in seen:   # distinct band sets (here: per k-point and side)
                seen.add((k, nb))
                ent += nb * ((cr.mill[k].shape[0] + 1 + 15) // 16 * 16)
    assert sizes["bf16"] <= 4 * ent
    # chi0: grows with the transitions and is the same for xo_chi0's single item
    w = np.array([0.0, 0.5, 1.0, 2.0])
    def item(nt, ng, prec, check=0):
        a = xo.Chi0Args()
        a.nt, a.ng, a.nw, a.prec = nt, ng, 4, xo.PREC[prec]
        a.rho, a.dE, a.chi0 = 8, 8, 8
        a.w, a.pref, a.check_dE = w.ctypes.data_as(C.POINTER(C.c_double)), 1.0, check
        return a
    for prec in ("fp64", "bf16x3"):
        small = xo.chi0_workspace_size([item(1000, 100, prec)])
        big = xo.chi0_workspace_size([item(50000, 100, prec)])
        assert 0 < small <= big
        assert xo.chi0_workspace_size([item(1000, 100, prec, check=1)]) == small + 256
        assert xo.chi0_workspace_size([item(1000, 100, prec), item(3000, 300, prec)]) > big * 0 + small
    # epsinv: pivot flags and scales, plus the saved column panel [nw][ng][64] complex128 past one block
    # (the flags and the per-frequency scale of the pivot test take 256 bytes each at this nw)
    assert xo.epsinv_workspace_size(64, 3) == 512
    assert xo.epsinv_workspace_size(400, 8) == 512 + 8 * 400 * 64 * 16
    with pytest.raises(xo.XoError):
        xo.epsinv_workspace_size(0, 1)


def test_autotune_rejects_accumulating_items():
    L = xo.lib()
    w = np.array([0.0, 1.0])
    a = xo.Chi0Args()
    a.nt, a.ng, a.nw, a.prec = 64, 16, 2, xo.PREC["bf16"]
    a.rho, a.dE, a.chi0 = 8, 8, 8
    a.w, a.pref, a.accumulate = w.ctypes.data_as(C.POINTER(C.c_double)), 1.0, 1
    best = xo.Tune()
    ms = C.c_double(0)
    rc = L.xo_chi0_autotune(C.byref(a), 1, C.byref(best), C.byref(ms), None)
    assert rc == xo.XO_ERR_ARG and b"accumulate" in L.xo_last_error()


def test_tail_predict_argument_errors():
    L = xo.lib()
    a = xo.TailPredictArgs()
    rc, msg = _rc(L.xo_tail_predict, a)
    assert rc == xo.XO_ERR_ARG and "null" in msg
    f64 = np.zeros(9)
    f32 = np.zeros(9, np.float32)
    m = np.zeros((3, 3), np.int32)
    a.chi_t = a.chi_h = a.params = a.Y = a.stats = 8   # never dereferenced: validation fails first
    a.qpg = a.bvec = a.w = f64.ctypes.data_as(C.POINTER(C.c_double))
    a.mill_g = m.ctypes.data_as(C.POINTER(C.c_int32))
    a.mu = a.isd = a.lo = a.hi = f32.ctypes.data_as(C.POINTER(C.c_float))
    dims = np.array([9, 256, 256, 256, 2], np.int32)
    a.dims = dims.ctypes.data_as(C.POINTER(C.c_int))
    a.ng, a.nw, a.nl, a.nmem = 3, 1, 4, 3
    rc, msg = _rc(L.xo_tail_predict, a)
    assert rc == xo.XO_ERR_ARG and "nmem" in msg
    a.nmem = 2
    dims[2] = 128                       # hidden widths other than 256
    rc, msg = _rc(L.xo_tail_predict, a)
    assert rc == xo.XO_ERR_UNSUPPORTED and "256" in msg
    dims[2], dims[0] = 256, 8           # not the 9 tail features
    rc, msg = _rc(L.xo_tail_predict, a)
    assert rc == xo.XO_ERR_UNSUPPORTED and "9" in msg
    dims[0] = 9
    a.nl = 6                            # more than three hidden 256 -> 256 layers
    rc, msg = _rc(L.xo_tail_predict, a)
    assert rc == xo.XO_ERR_ARG


def test_xterm_rejects_unknown_precision():
    L = xo.lib()
    a = xo.XtermArgs()
    mv = np.zeros((1, 3), np.int32)
    w = np.array([0.5])
    a.npw_v, a.nv, a.ng, a.nw, a.nn = 1, 1, 1, 1, 1
    a.mill_v = a.mill_g = mv.ctypes.data_as(C.POINTER(C.c_int32))
    a.w = w.ctypes.data_as(C.POINTER(C.c_double))
    a.coef_v = a.e_v = a.rho = a.out = 8   # never dereferenced: validation fails first
    a.pref, a.ebar = 1.0, 1.0
    a.prec = 9
    rc, msg = _rc(L.xo_xterm, a)
    assert rc == xo.XO_ERR_ARG and "precision" in msg

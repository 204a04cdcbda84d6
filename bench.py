#!/usr/bin/env python
"""Benchmark of the chi0 / eps^-1 hot path on one MI355X.

Default workload (the large cell): simple-cubic 2a supercell with 32 displaced fcc
sites, 2x2x2 k-points, q = b1/2, 128 occupied + 2000 empty bands, 72^3 FFT grid,
NG = 3000, 16 imaginary frequencies; K = 2 048 000 transitions. One step is the whole
path on inputs already resident in HBM: oscillator strengths for all 8 k-pairs
(xo_rho_batch), chi0 for all frequencies (xo_chi0) and the FP64 Dyson inversion
(xo_epsinv). The positive-definiteness flags of the inversion go to a device array and
are checked once after the timed steps, so the host enqueues the next step while the
GPU inverts.

Reported form: split bf16 ("bf16x3": operands split into bf16 hi + lo, three MFMA
products, FP32 accumulation over transition slices of at most 65 536 and FP64 across
slices), with the q -> 0 head and eps^-1 in FP64. The plain FP64 path is timed once in
the same run; its eps~^-1 is the error reference (e_F_vs_fp64, relative Frobenius,
worst frequency) and its step time gives speedup_vs_fp64. Plain bf16 (operands rounded
to bf16, one product) is timed beside it for reference only.

Each form runs its warm-up steps, the timed steps (HIP events at the stage boundaries
only) and then a few steps with the library's per-kernel HIP event brackets on
(xo_timing_enable), which give the kernel durations of the roofline entries without
weighing on the timed steps.

cpu_baseline: the FP64 oracle on the host cores, timed on a sample of the same workload
(one k-pair, a band subset, four frequencies, eps~^-1 of two) and extrapolated linearly in
the transitions and frequencies, which is exact for this work.

Other workloads (--workload): c2 (fcc 4x4x4 k, NG = 400: every form), c3 (27 q-points with
uneven G-sets in one batched launch), sigma (plasmon-pole W and the GW self-energy of
eight states summed over all 64 q of the c2 crystal), real (the c2 path at 100 real
frequencies); each prints its own JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp64_mfma": 78.6e12, "fp32_mfma": 157.3e12, "bf16_mfma": 2.5e15,
    "valu": 78.6e12,   # fp64 vector; fp32 vector without packed-FP32 instructions
}
GATE = 1e-4
MFMA_PEAK = {"fp64": PEAK["fp64_mfma"], "fp32": PEAK["fp32_mfma"], "bf16x3": PEAK["bf16_mfma"],
             "bf16": PEAK["bf16_mfma"]}
DTYPE = {"fp64": "f64", "fp32": "f32 (eps^-1 f64)", "bf16x3": "bf16x3+f32 (eps^-1 f64)",
         "bf16": "bf16+f32 (eps^-1 f64)"}


def chi0_flops(K, ng, nw):
    """Algorithmic chi0 flops: Hermitian half of a complex rank-K update, 8 flops/MAC."""
    return 4.0 * ng * ng * K * nw


def rho_direct_terms(cr):
    """Nonzero terms of the direct plane-wave sum, summed over the k-pairs: for each pair
    the (a, G) with a in the conduction sphere and a - (m_G - G0) in the valence sphere,
    times nc * nv. Each term is one complex multiply-add (8 flops)."""
    tot = 0
    G = cr.gmill.astype(np.int64)
    for ik, ikp, g0 in cr.pairs:
        mc, mv = cr.mill[ik].astype(np.int64), cr.mill[ikp].astype(np.int64)
        lo = mv.min(0)
        box = np.zeros(tuple(mv.max(0) - lo + 1), dtype=bool)
        box[tuple((mv - lo).T)] = True
        d = mc[:, None, :] - (G - np.asarray(g0))[None, :, :] - lo
        ok = np.all((d >= 0) & (d < np.array(box.shape)), axis=-1)
        hit = np.zeros(ok.shape, dtype=bool)
        hit[ok] = box[tuple(d[ok].T)]
        nc = cr.coef[ik].shape[0] - cr.nocc_at(ik)
        tot += int(hit.sum()) * nc * cr.nocc_at(ikp)
    return tot


def rho_zy_flops(cr, pairs_meta):
    """Useful flops of the rho_zy kernel per transition (stages 1 and 2, no padding).

    Stage 1: for every (x, y) the z-correlation sum_m conj(A(m)) B(m - e) over the
    overlap of the two z-spectra, for each needed e_z. Stage 2: the pruned y-DFT,
    Ny terms per needed (e_y, e_z) pair and x-plane. 8 real flops per complex MAC.
    """
    Nx, Ny, _ = cr.grid
    ik, ikp, g0 = pairs_meta
    mc, mv = cr.mill[ik], cr.mill[ikp]
    e = cr.gmill.astype(np.int64) - g0[None, :]
    cz = np.arange(mc[:, 2].min(), mc[:, 2].max() + 1)
    vz = set(range(mv[:, 2].min(), mv[:, 2].max() + 1))
    ez = range(e[:, 2].min(), e[:, 2].max() + 1)
    s1 = sum(sum(1 for m in cz if (m - ez_) in vz) for ez_ in ez)
    nyz = len({(int(a) % Ny, int(b)) for a, b in zip(e[:, 1], e[:, 2])})
    return 8.0 * Nx * (Ny * s1 + nyz * Ny)


def run_form(cr, prec, steps, warmup, ref_E=None, real=None, kernel_steps=None, keep_E=True):
    """One form of the path on crystal cr; real = (frequencies, eta) runs it at real frequencies
    (xo_chi0_real, Dyson step with the LU fallback) instead of the crystal's imaginary ones.
    kernel_steps: steps of the per-kernel timing pass (default: as many as timed)."""
    import torch
    from paper_1902_03837_amd import xo
    from paper_1902_03837_amd.pipeline import DeviceCrystal, rho_all, ntrans, CDTYPE, chi0_pref, qpg as qpg_of

    dc = DeviceCrystal.upload(cr, prec)
    ng, nw = cr.gmill.shape[0], len(cr.omegas) if real is None else len(real[0])
    K = ntrans(cr)
    dev = dc.coef[0].device
    M = torch.empty((K, ng), dtype=CDTYPE[prec], device=dev)
    dE = torch.empty(K, dtype=torch.float64, device=dev)
    chi = torch.empty((nw, ng, ng), dtype=torch.complex128, device=dev)
    E = torch.empty_like(chi)
    info = torch.zeros(nw, dtype=torch.int32, device=dev)   # pivot flags, read after the timed steps
    qpg = qpg_of(cr)
    pref = chi0_pref(cr)
    st = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(st)
        rho_all(dc, M, dE)
        if ev:
            ev[1].record(st)
        if real is None:
            xo.chi0(M, dE, cr.omegas, pref, out=chi, prec=prec, check_dE=False)
        else:
            xo.chi0_real(M, dE, real[0], real[1], pref, out=chi, prec=prec, check_dE=False)
        if ev:
            ev[2].record(st)
        xo.epsinv(chi, qpg, out=E, info=info, flags=xo.XO_EPS_SYM if real is None else xo.XO_EPS_LU_FALLBACK)
        if ev:
            ev[3].record(st)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # timed region: the library's per-kernel event brackets off, stage events only
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    # steps again with every kernel bracketed by HIP events on its launch stream
    ksteps = steps if kernel_steps is None else kernel_steps
    kern = {}
    if ksteps > 0:
        xo.timing_report()            # drop anything recorded before
        xo.timing_enable(True)
        for i in range(ksteps):
            step()
        torch.cuda.synchronize()
        xo.timing_enable(False)
        kern = xo.timing_report()
    if int(info.abs().sum().item()):
        raise RuntimeError(f"eps~ inversion failed ({prec}): pivot flags {info.tolist()}")
    stages = np.array([[evs[i][j].elapsed_time(evs[i][j + 1]) for j in range(3)] for i in range(steps)])
    step_ms = np.array([evs[i][0].elapsed_time(evs[i][3]) for i in range(steps)])
    out = dict(prec=prec, K=K, ms_per_step=float(np.median(step_ms)), wall_ms_per_step=wall * 1e3,
               t_rho_ms=float(np.median(stages[:, 0])), t_chi0_ms=float(np.median(stages[:, 1])),
               t_eps_ms=float(np.median(stages[:, 2])),
               kernels={k: dict(launches=v[0] // max(1, ksteps), ms_per_step=v[1] / max(1, ksteps),
                                avg_launch_ms=v[1] / v[0]) for k, v in kern.items()})
    E_host = E.cpu().numpy() if keep_E or ref_E is not None else None
    if ref_E is not None:
        from_ref = [float(np.linalg.norm(E_host[j] - ref_E[j]) / np.linalg.norm(ref_E[j])) for j in range(nw)]
        out["e_F_vs_fp64"] = max(from_ref)
    del M, dE, chi, E, dc
    torch.cuda.empty_cache()
    return out, E_host


def cpu_baseline(cr, npairs):
    """The FP64 oracle as it stands, on the host cores, for the first npairs k-pairs."""
    from oracle.pipeline import rho_pair
    from oracle.chi0 import chi0_from_rho, crystal_prefactor
    from oracle.epsinv import epsinv_sym, crystal_qpg
    t0 = time.perf_counter()
    Ms, ds = [], []
    for ip in range(npairs):
        m, d = rho_pair(cr, ip, "fft")
        Ms.append(m)
        ds.append(d)
    M, dE = np.concatenate(Ms), np.concatenate(ds)
    chi = chi0_from_rho(M, dE, cr.omegas, crystal_prefactor(cr))
    epsinv_sym(chi, crystal_qpg(cr), check=False)
    dt = time.perf_counter() - t0
    ng, nw = cr.gmill.shape[0], len(cr.omegas)
    K = M.shape[0]
    return dict(value=chi0_flops(K, ng, nw) / dt / 1e9, unit="GFLOP/s", cores=len(os.sched_getaffinity(0)),
                kind="oracle", seconds=dt, transitions_per_s_per_qw=K * nw / dt,
                sample=f"{npairs} of {len(cr.pairs)} k-pairs (K={K} transitions), full NG and frequencies; "
                       f"numpy FFT single-threaded, BLAS on all cores")


def measured_traffic(kernel, summary="c2_hbm_traffic.txt"):
    """HBM bytes per launch (read + write) from a committed counter summary, or None.

    Only used when the kernel's source file still has the hash recorded with the
    counters; otherwise the figures describe an older kernel and are not reported.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    src, tr = {}, {}
    for line in open(path):
        f = line.split()
        if len(f) == 4 and f[0] == "source":
            src[f[1]] = (f[2], f[3])
        elif len(f) == 4 and f[0] == "traffic_GB":
            tr[f[1]] = (float(f[2]) + float(f[3])) * 1e9
    if kernel not in src or kernel not in tr:
        return None
    fname, h = src[kernel]
    cur = hashlib.sha256(open(os.path.join(ROOT, fname), "rb").read()).hexdigest()[:16]
    return tr[kernel] if cur == h else None


def roofline(cr, form, K, nw, ng, name=None, summary="c2_hbm_traffic.txt"):
    """Roofline entry of one kernel (default: the one with the largest time per step); traffic
    comes from the committed counter summary of the workload while the kernel source is unchanged."""
    kern = form["kernels"]
    if name is None:
        name = max(kern, key=lambda k: kern[k]["ms_per_step"])
    k = kern[name]
    t = k["avg_launch_ms"] * 1e-3
    prec = form["prec"]
    if name.startswith("chi0_tiles") or name.startswith("chi0_blocks"):
        # one launch covers every frequency group of the call (imaginary axis)
        fl = chi0_flops(K, ng, nw)
        peak = MFMA_PEAK[prec]
        return dict(kernel=name, bound="mfma", achieved=fl / t / 1e12, peak=peak / 1e12, unit="TFLOP/s",
                    frac=fl / t / peak, traffic=measured_traffic(name, summary),
                    note="algorithmic flops 4 NG^2 K per frequency (Hermitian half)")
    if name == "rho_zy":
        per_t = np.mean([rho_zy_flops(cr, p) for p in cr.pairs])
        units = K / k["launches"]                   # transitions per launch (one k-pair)
        fl = per_t * units
        return dict(kernel=name, bound="alu", achieved=fl / t / 1e12, peak=PEAK["valu"] / 1e12,
                    unit="TFLOP/s", frac=fl / t / PEAK["valu"], traffic=None,
                    note="useful complex MACs of the z-correlation and pruned y-DFT, 8 flops each")
    if name.startswith("rho_gemm"):
        fl = 8.0 * rho_direct_terms(cr) / k["launches"]   # per launch (all pairs of the step in one)
        peak = MFMA_PEAK[prec]
        return dict(kernel=name, bound="mfma", achieved=fl / t / 1e12, peak=peak / 1e12,
                    unit="TFLOP/s", frac=fl / t / peak, traffic=measured_traffic(name, summary),
                    note="algorithmic flops: the nonzero terms of the direct plane-wave sum (8 per complex "
                         "multiply-add) over the dense MFMA peak of the precision; the kernel also executes "
                         "the zero terms of its dense tiles" + (" and three split-bf16 products per term"
                                                                 if prec == "bf16x3" else ""))
    if name == "rho_yz":
        # algorithmic count: an FFT of the product grid per transition, 5 N_r log2 N_r
        nr = float(np.prod(cr.grid))
        fl = 5.0 * nr * np.log2(nr) * K / k["launches"]
        return dict(kernel=name, bound="mfma", achieved=fl / t / 1e12, peak=PEAK["bf16_mfma"] / 1e12,
                    unit="TFLOP/s", frac=fl / t / PEAK["bf16_mfma"], traffic=measured_traffic(name, summary),
                    note="algorithmic flops 5 N_r log2 N_r per transition (FFT-equivalent) over the bf16 "
                         "dense peak; the kernel executes the y-z correlation as split-bf16 (x3) 16x16x32 tiles")
    return dict(kernel=name, bound="unknown", achieved=None, peak=None, unit=None, frac=None, traffic=None)


def cpu_baseline_sampled(cr, nv_s=16, nc_s=192, nw_s=4, nw_eps=2):
    """The FP64 oracle as it stands on the host cores, on a sample of the workload: rho of
    nv_s x nc_s transitions of the first k-pair (FFT route), chi0 of those at nw_s frequencies
    (zgemm), eps~^-1 at nw_eps frequencies. Each stage is timed and scaled linearly to the
    whole step (rho and chi0 with the transitions, chi0 and eps~^-1 with the frequencies)."""
    from oracle.rho import rho_fft
    from oracle.chi0 import chi0_from_rho, crystal_prefactor
    from oracle.epsinv import epsinv_sym, crystal_qpg
    ik, ikp, g0 = cr.pairs[0]
    nv = cr.nocc_at(ikp)
    cc = cr.coef[ik][cr.nocc_at(ik):cr.nocc_at(ik) + nc_s]
    cv = cr.coef[ikp][:nv_s]
    t0 = time.perf_counter()
    r = rho_fft(cc, cr.mill[ik], cv, cr.mill[ikp], cr.gmill, g0, cr.grid)
    t1 = time.perf_counter()
    M = r.reshape(-1, r.shape[-1])
    dE = (cr.eps[ik][cr.nocc_at(ik):cr.nocc_at(ik) + nc_s][None, :] - cr.eps[ikp][:nv_s][:, None]).reshape(-1)
    chi = chi0_from_rho(M, dE, cr.omegas[:nw_s], crystal_prefactor(cr))
    t2 = time.perf_counter()
    epsinv_sym(chi[:nw_eps], crystal_qpg(cr), check=False)
    t3 = time.perf_counter()
    K = sum((cr.coef[a].shape[0] - cr.nocc_at(a)) * cr.nocc_at(b) for a, b, _ in cr.pairs)
    ks, nw = M.shape[0], len(cr.omegas)
    t_full = (t1 - t0) * K / ks + (t2 - t1) * (K / ks) * (nw / nw_s) + (t3 - t2) * nw / nw_eps
    ng = cr.gmill.shape[0]
    return dict(value=chi0_flops(K, ng, nw) / t_full / 1e9, unit="GFLOP/s", cores=len(os.sched_getaffinity(0)),
                kind="oracle", extrapolated=True, seconds_sampled=t3 - t0, seconds_extrapolated_step=t_full,
                transitions_per_s_per_qw=K * nw / t_full,
                sample=f"k-pair 0: {nv_s} valence x {nc_s} conduction bands ({ks} of {K} transitions), rho by "
                       f"the FFT route ({t1 - t0:.1f} s), chi0 at {nw_s} of {nw} frequencies ({t2 - t1:.1f} s), "
                       f"eps~^-1 at {nw_eps} ({t3 - t2:.1f} s); scaled linearly in transitions and frequencies; "
                       f"scipy.fft on all cores, BLAS threads as set for the process")


def copy_calibration():
    """A 1 GiB device-to-device copy: the reference launch for scaling the HBM counters."""
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    return 2 * a.numel() * 8


def roofline_eps(kern, ng, nw):
    """Roofline of the eps~^-1 rank update on FP64 matrix cores (rank_update_mfma): algorithmic
    flops 8 (NG - kb)^2 kb per 64-wide block column and frequency (the complex multiply-adds of the
    entries outside the block's rows and columns, Eq. X_rpa_inv by Gauss-Jordan), over the kernel's
    event-timed time per step, against the FP64 matrix-core peak."""
    k = kern.get("eps_rank_update")
    if not k:
        return None
    fl = 0.0
    for k0 in range(0, ng, 64):
        kb = min(64, ng - k0)
        fl += 8.0 * (ng - kb) ** 2 * kb
    ach = fl * nw / (k["ms_per_step"] / 1e3) / 1e12
    peak = PEAK["fp64_mfma"] / 1e12
    return {"kernel": "rank_update_mfma", "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
            "frac": ach / peak, "traffic": None,
            "note": "algorithmic FP64 flops 8 (NG - kb)^2 kb per block column and frequency"}


def run_c5(args):
    """Headline: the large cell (32-site simple-cubic supercell, 2x2x2 k, q = b1/2, 128 occupied +
    2000 empty bands, 72^3 grid, NG = 3000, 16 frequencies, K = 2 048 000) in the split-bf16 form,
    the plain FP64 path once for the error of eps~^-1 and the speedup."""
    import torch
    from synth.cache import cached_crystal
    t0 = time.perf_counter()
    cr = cached_crystal("c5", args.fixture_cache,
                        progress=lambda m: print(f"[bench] c5 fixture {m}", file=sys.stderr, flush=True))
    t_fix = time.perf_counter() - t0
    ng, nw = cr.gmill.shape[0], len(cr.omegas)
    print(f"[bench] c5 fixture ready in {t_fix:.1f} s", file=sys.stderr, flush=True)
    form = args.c5_form
    kst = max(1, args.kernel_steps)
    res_form, E = run_form(cr, form, args.steps, args.warmup, kernel_steps=kst)
    print(f"[bench] c5 {form}: {res_form['ms_per_step']:.1f} ms/step (rho {res_form['t_rho_ms']:.1f}, chi0 "
          f"{res_form['t_chi0_ms']:.1f}, eps {res_form['t_eps_ms']:.1f})", file=sys.stderr, flush=True)
    others = {}
    for p in [x for x in args.c5_beside.split(",") if x and x != form]:
        r, _ = run_form(cr, p, min(args.steps, 3), 1, kernel_steps=1, keep_E=False)
        others[p] = r
        print(f"[bench] c5 {p} (beside): {r['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64, E64 = run_form(cr, "fp64", 1, 1, kernel_steps=1)
        print(f"[bench] c5 fp64: {r64['ms_per_step']:.1f} ms/step (rho {r64['t_rho_ms']:.1f}, chi0 "
              f"{r64['t_chi0_ms']:.1f}, eps {r64['t_eps_ms']:.1f})", file=sys.stderr, flush=True)
        res_form["e_F_vs_fp64"] = max(float(np.linalg.norm(E[j] - E64[j]) / np.linalg.norm(E64[j]))
                                      for j in range(nw))
        res_form["e_S_vs_fp64"] = max(float(np.linalg.norm(E[j] - E64[j]) / np.linalg.norm(E64[j] - np.eye(ng)))
                                      for j in range(nw))
        res_form["e_head_vs_fp64"] = max(float(abs(E[j, 0, 0] - E64[j, 0, 0]) / abs(E64[j, 0, 0]))
                                         for j in range(nw))
        del E64
        print(f"[bench] c5 {form}: e_F vs fp64 {res_form['e_F_vs_fp64']:.2e}", file=sys.stderr, flush=True)
    del E
    K = res_form["K"]
    t = res_form["ms_per_step"] * 1e-3
    fl = chi0_flops(K, ng, nw)
    res = {
        "metric": "chi0 GFLOP/s + transitions/s per q,w; speedup vs FP64 at eps^-1 rel err<=1e-4",
        "value": fl / t / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res_form["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[form],
        "data": "synthetic",
        "config": {"workload": f"c5: sc 2a supercell (32 displaced fcc sites), 2x2x2 k, q = b1/2, 128 occ + "
                               f"2000 empty bands, FFT 72^3, NG={ng}, {nw} imaginary frequencies, K={K} "
                               f"transitions",
                   "form": form, "global_batch": K, "parallelism": "single GPU"},
        "transitions_per_s_per_qw": K * nw / t,
        "speedup_vs_fp64": (r64["ms_per_step"] / res_form["ms_per_step"]) if r64 else None,
        "e_F_vs_fp64": res_form.get("e_F_vs_fp64"),
        "e_S_vs_fp64": res_form.get("e_S_vs_fp64"),
        "gate": GATE,
        "stage_ms": {"rho": res_form["t_rho_ms"], "chi0": res_form["t_chi0_ms"], "eps": res_form["t_eps_ms"]},
        "fp64_ms_per_step": r64["ms_per_step"] if r64 else None,
        "full_matrix_equivalent_GFLOPs": 2 * fl / t / 1e9,
        "roofline": roofline(cr, res_form, K, nw, ng, summary="c5_hbm_traffic.txt"),
        "fixture_s": t_fix,
        "kernels_ms_per_step": {k: v["ms_per_step"] for k, v in res_form["kernels"].items()},
    }
    rk = [k for k in res_form["kernels"] if k.startswith("rho_gemm") or k in ("rho_yz", "rho_zy")]
    if rk and rk[0] != res["roofline"]["kernel"]:
        res["roofline_rho"] = roofline(cr, res_form, K, nw, ng, name=rk[0], summary="c5_hbm_traffic.txt")
    res["roofline_eps"] = roofline_eps(res_form["kernels"], ng, nw)
    res["beside"] = {p: dict(ms_per_step=r["ms_per_step"], stage_ms={"rho": r["t_rho_ms"], "chi0": r["t_chi0_ms"],
                                                                      "eps": r["t_eps_ms"]},
                             note="timed for reference, not the reported form")
                     for p, r in others.items()}
    if r64:
        res["roofline_fp64"] = roofline(cr, r64, K, nw, ng, name=next(
            k for k in r64["kernels"] if k.startswith("chi0_tiles")), summary="c5_hbm_traffic.txt")
    if not args.no_cpu:
        print("[bench] timing the oracle on the host cores (sampled)", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline_sampled(cr)
    if args.copy_calibration:
        res["copy_calibration_bytes"] = copy_calibration()
    if args.detail:
        with open(args.detail, "w") as fh:
            json.dump(dict(result=res, form=res_form, fp64=r64, beside=others), fh, indent=1)
    print(json.dumps(res), flush=True)


def run_c3(args):
    """Batched persistent workload: 3x3x3 k-grid, all 27 q-points, uneven G-sets (169..893),
    32 occupied + 400 empty bands, 48^3 grid, 16 frequencies; bf16 (plain and split) rho and
    chi0 with one persistent chi0 launch over all q (tiles autotuned), FP64 eps^-1 per q."""
    import torch
    from synth.configs import crystal_q_set
    from paper_1902_03837_amd import xo, tune
    from paper_1902_03837_amd.pipeline import DeviceCrystal, rho_all, ntrans, CDTYPE, chi0_pref, qpg

    t0 = time.perf_counter()
    crs = crystal_q_set("c3", nq=args.nq)
    t_fix = time.perf_counter() - t0
    print(f"[bench] c3 fixture: {len(crs)} q-points, NG {[c.gmill.shape[0] for c in crs]}, {t_fix:.1f} s",
          file=sys.stderr, flush=True)
    nw = len(crs[0].omegas)

    def build(prec):
        base = DeviceCrystal.upload(crs[0], prec)
        dcs = [DeviceCrystal(cr, prec, base.coef, base.eps) for cr in crs]
        bufs = []
        for cr in crs:
            ng, K = cr.gmill.shape[0], ntrans(cr)
            bufs.append(dict(M=torch.empty((K, ng), dtype=CDTYPE[prec], device="cuda"),
                             dE=torch.empty(K, dtype=torch.float64, device="cuda"),
                             chi=torch.empty((nw, ng, ng), dtype=torch.complex128, device="cuda"),
                             E=torch.empty((nw, ng, ng), dtype=torch.complex128, device="cuda"),
                             info=torch.zeros(nw, dtype=torch.int32, device="cuda")))
        return dcs, bufs

    # the q-points' inversions are independent: four streams (default priority) overlap
    # their latency-bound block chains
    side = [torch.cuda.Stream() for _ in range(4)]

    def step(dcs, bufs, prec, tn, ev=None):
        st = torch.cuda.current_stream()
        if ev:
            ev[0].record(st)
        for dc, b in zip(dcs, bufs):
            rho_all(dc, b["M"], b["dE"])
        if ev:
            ev[1].record(st)
        xo.chi0_batch([(b["M"], b["dE"], chi0_pref(dc.cr), b["chi"]) for dc, b in zip(dcs, bufs)], crs[0].omegas,
                      prec=prec, tune=tn, check_dE=False)
        if ev:
            ev[2].record(st)
        for sd in side:
            sd.wait_stream(st)
        for j, (dc, b) in enumerate(zip(dcs, bufs)):
            xo.epsinv(b["chi"], qpg(dc.cr), out=b["E"], info=b["info"], stream=side[j % len(side)])
        for sd in side:
            st.wait_stream(sd)
        if ev:
            ev[3].record(st)

    out = {}
    Eall = {}
    for prec in args.c3_forms.split(","):
        dcs, bufs = build(prec)
        tn = None
        if prec != "fp64":
            for dc, b in zip(dcs, bufs):
                rho_all(dc, b["M"], b["dE"])
            items = [(b["M"], b["dE"], chi0_pref(dc.cr), b["chi"]) for dc, b in zip(dcs, bufs)]
            tn, tms, cached = tune.tuned(items, crs[0].omegas, prec, path=args.tune_cache)
            print(f"[bench] c3 {prec}: tuned chi0 launch {tn} ({tms:.2f} ms on a sample, cached={cached})",
                  file=sys.stderr, flush=True)
        nsteps = args.steps if prec != "fp64" else 1
        for _ in range(args.warmup if prec != "fp64" else 0):
            step(dcs, bufs, prec, tn)
        torch.cuda.synchronize()
        xo.timing_report()
        xo.timing_enable(True)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(nsteps)]
        for i in range(nsteps):
            step(dcs, bufs, prec, tn, evs[i])
        torch.cuda.synchronize()
        xo.timing_enable(False)
        kern = xo.timing_report()
        if any(int(b["info"].abs().sum().item()) for b in bufs):
            raise RuntimeError(f"eps~ not positive definite at some q ({prec})")
        ms = float(np.median([evs[i][0].elapsed_time(evs[i][3]) for i in range(nsteps)]))
        st = [float(np.median([evs[i][j].elapsed_time(evs[i][j + 1]) for i in range(nsteps)])) for j in range(3)]
        Ks = [b["M"].shape[0] for b in bufs]
        ngs = [b["M"].shape[1] for b in bufs]
        fl = sum(4.0 * ng * ng * K * nw for ng, K in zip(ngs, Ks))
        res = dict(ms_per_step=ms, stage_ms=dict(rho=st[0], chi0=st[1], eps=st[2]),
                   chi0_GFLOPs=fl / (ms * 1e-3) / 1e9, chi0_kernel_TFLOPs=None,
                   transitions_per_s_per_qw=sum(Ks) * nw / (ms * 1e-3), tune=tn,
                   kernels={k: dict(launches=v[0] // nsteps, ms_per_step=v[1] / nsteps) for k, v in kern.items()})
        ck = [k for k in kern if k.startswith("chi0_tiles") or k.startswith("chi0_blocks")]
        if ck:
            res["chi0_kernel_TFLOPs"] = fl / (kern[ck[0]][1] / nsteps * 1e-3) / 1e12
        Eall[prec] = [b["E"].cpu().numpy() for b in bufs]
        out[prec] = res
        print(f"[bench] c3 {prec}: {ms:.1f} ms/step (rho {st[0]:.1f}, chi0 {st[1]:.1f}, eps {st[2]:.1f}), "
              f"chi0 {res['chi0_GFLOPs']:.0f} GFLOP/s over the step", file=sys.stderr, flush=True)
        del dcs, bufs
        torch.cuda.empty_cache()
    if "fp64" in Eall:
        for prec in out:
            if prec != "fp64":
                out[prec]["e_F_vs_fp64"] = max(float(np.linalg.norm(E[j] - R[j]) / np.linalg.norm(R[j]))
                                               for E, R in zip(Eall[prec], Eall["fp64"]) for j in range(nw))
                print(f"[bench] c3 {prec}: e_F vs fp64 {out[prec]['e_F_vs_fp64']:.3e}", file=sys.stderr,
                      flush=True)
    res = {"metric": "chi0 GFLOP/s + transitions/s per q,w (batched persistent workload)",
           "workload": f"c3: fcc 3x3x3 k, {len(crs)} q-points, NG {min(c.gmill.shape[0] for c in crs)}.."
                       f"{max(c.gmill.shape[0] for c in crs)}, 32 occ + 400 empty bands, FFT 48^3, {nw} freqs",
           "forms": out, "fixture_s": t_fix}
    if args.detail:
        with open(args.detail, "w") as fh:
            json.dump(res, fh, indent=1)
    print(json.dumps(res), flush=True)


def sigma_flops(ng, nb, nn, nz):
    """Algorithmic FP64 flops of one xo_sigma launch (Sigma_c part): per (G, G', m, n) the
    product rho(G) conj(rho(G')) Wr (two complex multiplies, 12 flops), per frequency the
    complex denominator (2), its squared modulus (3), one reciprocal (1), the product with the
    conjugate denominator (6), the scaling (2) and the accumulation (2): 16 flops."""
    return float(ng) * ng * nb * nn * (12 + 16 * nz)


def run_sigma(args):
    """GW self-energy of eight states around the gap at Gamma on the c2 crystal (fcc 4x4x4 k,
    16 occupied + 200 empty bands, NG = 400): per q (all 64) the oscillator strengths of the
    states against all 216 bands at k - q (xo_rho, FP64), the plasmon-pole fit of eps~^-1 at
    0 and i 1 Ha (xo_ppa_fit) and Sigma_x plus Sigma_c at three frequencies per state
    (xo_sigma). eps~^-1 of every q is made by the library's FP64 path before the timed steps."""
    import dataclasses
    import torch
    from synth import crystal_for
    from synth.crystal import find_pairs, alias_extents
    from paper_1902_03837_amd import xo
    from paper_1902_03837_amd.pipeline import DeviceCrystal, run_crystal, ntrans, SigmaPlan, sigma_kpoint
    t0 = time.perf_counter()
    base = dataclasses.replace(crystal_for("c2"), omegas=np.array([0.0, 1.0]))
    crs = []
    for q in base.kf:
        cr = dataclasses.replace(base, qf=q.copy(), pairs=find_pairs(base.kf, q))
        for ik, ikp, g0 in cr.pairs:
            if np.any(alias_extents(cr.grid, cr.mill[ik], cr.mill[ikp], cr.gmill, g0) >= np.array(cr.grid)):
                raise ValueError(f"q {q}: FFT grid aliases")
        crs.append(cr)
    t_fix = time.perf_counter() - t0
    print(f"[bench] sigma fixture: {len(crs)} q built in {t_fix:.1f} s", file=sys.stderr, flush=True)
    dc = DeviceCrystal.upload(base, "fp64")
    ng, nk = base.gmill.shape[0], base.nk
    K = ntrans(base)
    M = torch.empty((K, ng), dtype=torch.complex128, device="cuda")
    dE = torch.empty(K, dtype=torch.float64, device="cuda")
    chi = torch.empty((2, ng, ng), dtype=torch.complex128, device="cuda")
    t0 = time.perf_counter()
    Es = []
    for cr in crs:
        Es.append(run_crystal(DeviceCrystal(cr, "fp64", dc.coef, dc.eps), M=M, dE=dE, chi=chi)[3].clone())
    torch.cuda.synchronize()
    del M, dE, chi
    print(f"[bench] sigma: eps~^-1 of {len(crs)} q in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    nn, nz, eta = 8, 3, 0.01
    states = slice(base.nocc - nn // 2, base.nocc + nn // 2)
    z = np.stack([base.eps[0][states] + d for d in (-0.05, 0.0, 0.05)], axis=1).astype(np.complex128)
    zt = torch.from_numpy(z).cuda()
    plan = SigmaPlan(dc, crs, 0, states)
    sigc = torch.empty((nn, nz), dtype=torch.complex128, device="cuda")
    sigx = torch.empty((nn,), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        sigma_kpoint(plan, Es, zt, sigc, sigx, eta=eta)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        sigma_kpoint(plan, Es, zt, sigc, sigx, eta=eta)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    xo.timing_enable(True)
    for _ in range(args.steps):
        sigma_kpoint(plan, Es, zt, sigc, sigx, eta=eta)
    torch.cuda.synchronize()
    rep = xo.timing_report()
    xo.timing_enable(False)
    nb = base.coef[0].shape[0]
    fl_q = sigma_flops(ng, nb, nn, nz)
    kern = {k: {"calls": int(v[0]), "avg_ms": v[1] / v[0]} for k, v in rep.items()}
    ks = kern["sigma_c_tiles"]["avg_ms"] * 1e-3
    ach = fl_q / ks / 1e12
    gx, gc = sigx.cpu().numpy(), sigc.cpu().numpy()
    print(f"[bench] sigma: {ms:.2f} ms/step; sigma_c_tiles {ks * 1e3:.3f} ms/launch = {ach:.1f} TFLOP/s; "
          f"Sigma_x {np.round(gx, 4)}; Sigma_c(e_n) {np.round(gc[:, 1], 4)}", file=sys.stderr, flush=True)
    res = {"metric": "GW self-energy matrix elements per second (states x frequencies x q)",
           "value": nn * nz * len(crs) / (ms * 1e-3), "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"sigma: c2 crystal (fcc 4x4x4 k, 16 occ + 200 empty bands, NG={ng}), "
                                  f"{nn} states at Gamma, {nz} frequencies each, all {len(crs)} q, plasmon pole "
                                  f"from eps~^-1 at 0 and i 1 Ha", "parallelism": "single GPU"},
           "sigma_x": gx.tolist(), "sigma_c_at_e": [[c.real, c.imag] for c in gc[:, 1]],
           "kernels_ms_per_launch": {k: v["avg_ms"] for k, v in kern.items()},
           "roofline": {"kernel": "sigma_c_tiles", "bound": "alu", "achieved": ach, "peak": PEAK["valu"] / 1e12,
                        "unit": "TFLOP/s", "frac": ach * 1e12 / PEAK["valu"],
                        "traffic": measured_traffic("sigma_c_tiles", "sigma_hbm_traffic.txt"),
                        "note": "algorithmic FP64 flops per launch (ng^2 nb nn (12 + 16 nz), a reciprocal "
                                "counted as one) over the FP64 vector peak"}}
    if not args.no_cpu:
        import oracle.sigma as osig
        t0 = time.perf_counter()
        pick = [0, nn - 1]
        cr = crs[5]
        osig.sigma_kpoint([cr], [Es[5].cpu().numpy()], 0, [states.start + i for i in pick], z[pick], eta=eta)
        dt = time.perf_counter() - t0
        frac = len(pick) / nn / len(crs)
        res["cpu_baseline"] = {"value": nn * nz * len(crs) * frac / dt, "unit": "elements/s",
                               "cores": torch.get_num_threads(), "kind": "oracle",
                               "sample": f"one q of {len(crs)}, {len(pick)} of {nn} states ({dt:.1f} s)"}
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = 2 * a.numel() * 8
    print(json.dumps(res), flush=True)


def run_eps(args):
    """The eps~^-1 stage alone (Eq. X_rpa_inv, blocked Gauss-Jordan in FP64): for each NG x
    frequencies in --eps-sizes, a seeded synthetic chi0 = -0.05 B B^H / NG (B complex Gaussian,
    so eps~ is Hermitian positive definite, formed on the GPU) and |q+G| spread over [0.5, 3];
    the time per call (events over --steps calls after --warmup) and per kernel (the library's
    brackets over as many calls), and the rank update's matrix-core roofline."""
    import torch
    from paper_1902_03837_amd import xo
    sizes = []
    for tok in args.eps_sizes.split(","):
        a, b = tok.lower().split("x")
        sizes.append((int(a), int(b)))
    res = {}
    for ng, nw in sizes:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(ng * 1000 + nw)
        B = torch.randn((nw, ng, ng), dtype=torch.complex128, device="cuda", generator=gen) / np.sqrt(ng)
        chi = -torch.matmul(B, B.conj().transpose(-1, -2).contiguous()) * 0.05
        del B
        q = np.linspace(0.5, 3.0, ng)
        out = torch.empty_like(chi)
        info = torch.zeros(nw, dtype=torch.int32, device="cuda")
        for _ in range(args.warmup):
            xo.epsinv(chi, q, out=out, info=info)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            xo.epsinv(chi, q, out=out, info=info)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        xo.timing_report()
        xo.timing_enable(True)
        for _ in range(args.steps):
            xo.epsinv(chi, q, out=out, info=info)
        torch.cuda.synchronize()
        xo.timing_enable(False)
        kern = {name: {"launches_per_call": n / args.steps, "ms_per_call": t / args.steps, "avg_launch_ms": t / n}
                for name, (n, t) in xo.timing_report().items()}
        flags = int(info.max().item())
        if flags:
            raise SystemExit(f"bench.py: eps~ of NG={ng} not positive definite (flag {flags})")
        roof = roofline_eps({"eps_rank_update": {"ms_per_step": kern["eps_rank_update"]["ms_per_call"]}}, ng, nw) \
            if "eps_rank_update" in kern else None
        res[f"{ng}x{nw}"] = {"ng": ng, "nw": nw, "ms_per_call": ms, "kernels": kern, "roofline_rank_update": roof}
        print(f"[bench] eps NG={ng} x {nw}: {ms:.3f} ms per call", file=sys.stderr, flush=True)
        del chi, out
    first = res[f"{sizes[0][0]}x{sizes[0][1]}"]
    print(json.dumps({"metric": "eps~^-1 time per call (all frequencies)", "value": first["ms_per_call"], "unit": "ms",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": first["ms_per_call"],
                      "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                      "data": "synthetic",
                      "config": {"workload": "eps: seeded Hermitian positive definite eps~ at NG x frequencies "
                                             + ", ".join(f"{a} x {b}" for a, b in sizes),
                                 "parallelism": "single GPU"},
                      "sizes": res}), flush=True)


def run_real(args):
    """Real-axis workload: the c2 crystal (fcc 4x4x4 k, q = b1/4, 16 occupied + 200 empty bands,
    36^3, NG = 400, K = 204 800) at 100 real frequencies spread evenly over [0, max dE] with
    eta = 0.1 eV: rho, xo_chi0_real (two Hermitian weighted updates per frequency) and the
    Dyson step with the LU fallback; each form against plain FP64 timed in the same run."""
    from synth import crystal_for
    cr = crystal_for("c2")
    ng = cr.gmill.shape[0]
    dmax = max(float(np.max(cr.eps[ik][cr.nocc_at(ik):]) - np.min(cr.eps[ikp][:cr.nocc_at(ikp)]))
               for ik, ikp, _ in cr.pairs)
    ws = list(np.linspace(0.0, dmax, args.real_nw))
    eta = 0.1 / 27.211386
    out, Es = {}, {}
    forms = args.real_forms.split(",")
    for prec in [p for p in forms if p != "fp64"] + (["fp64"] if "fp64" in forms else []):
        steps, warm = (args.steps, args.warmup) if prec != "fp64" else (1, 1)
        r, Es[prec] = run_form(cr, prec, steps, warm, real=(ws, eta))
        print(f"[bench] real {prec}: {r['ms_per_step']:.1f} ms/step (rho {r['t_rho_ms']:.1f}, chi0 "
              f"{r['t_chi0_ms']:.1f}, eps {r['t_eps_ms']:.1f})", file=sys.stderr, flush=True)
        out[prec] = r
    K = next(iter(out.values()))["K"]
    nslot = 2 * len(ws)
    fl = chi0_flops(K, ng, nslot)   # two Hermitian updates per frequency
    for prec, r in out.items():
        if "fp64" in out and prec != "fp64":
            E64 = Es["fp64"]
            r["e_F_vs_fp64"] = max(float(np.linalg.norm(Es[prec][j] - E64[j]) / np.linalg.norm(E64[j]))
                                   for j in range(len(ws)))
            r["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / r["ms_per_step"]
        ck = [k for k in r["kernels"] if k.startswith("chi0_tiles") or k.startswith("chi0_blocks")]
        t = sum(r["kernels"][k]["ms_per_step"] for k in ck) * 1e-3
        r["chi0_kernel_TFLOPs"] = fl / t / 1e12
        r["chi0_kernel_frac_of_peak"] = fl / t / MFMA_PEAK[prec]
        print(f"[bench] real {prec}: chi0 kernels {t * 1e3:.1f} ms = {fl / t / 1e12:.1f} TFLOP/s; "
              f"e_F vs fp64 {r.get('e_F_vs_fp64')}", file=sys.stderr, flush=True)
    res = {"metric": "chi0 GFLOP/s at real frequencies; speedup vs FP64 at eps^-1 rel err<=1e-4",
           "workload": f"real: c2 crystal, {len(ws)} real frequencies on [0, {dmax:.3f}] Ha, eta = 0.1 eV, "
                       f"NG={ng}, K={K} transitions",
           "forms": out,
           "note": "chi0_kernel_frac_of_peak: algorithmic flops 4 NG^2 K per Hermitian update (two per "
                   "frequency: weights Re F and Im F) over the dense peak of the executed precision"}
    if args.detail:
        with open(args.detail, "w") as fh:
            json.dump(res, fh, indent=1)
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--forms", default="fp64,fp32,bf16x3,bf16")
    ap.add_argument("--cpu-pairs", type=int, default=6, help="k-pairs of the oracle's CPU timing (about 13 s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--detail", default=None, help="write the per-form detail JSON here")
    ap.add_argument("--nq", type=int, default=27, help="c3: number of q-points")
    ap.add_argument("--c3-forms", default="bf16,bf16x3,fp64", help="c3: forms to time (fp64 is the reference)")
    ap.add_argument("--tune-cache", default=None, help="c3: JSON file for autotuned launch shapes")
    ap.add_argument("--c5-form", default="bf16x3", help="c5: the reported form")
    ap.add_argument("--c5-beside", default="bf16", help="c5: forms timed beside it for reference (comma list)")
    ap.add_argument("--no-fp64", action="store_true", help="c5: skip the FP64 reference run")
    ap.add_argument("--kernel-steps", type=int, default=2, help="c5: steps of the per-kernel timing pass")
    ap.add_argument("--fixture-cache", default=None, help="directory to keep generated crystals in (npz)")
    ap.add_argument("--real-forms", default="bf16,bf16x3,fp64", help="real: forms (fp64 gives the error reference)")
    ap.add_argument("--real-nw", type=int, default=100, help="real: number of real frequencies")
    ap.add_argument("--eps-sizes", default="400x8,900x16,3000x16", help="eps: NGxfrequencies, comma list")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 1 GiB device-to-device copy (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for {args.gpus}); "
              "multi-GPU sharding is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    from synth import crystal_for

    if args.workload == "c3":
        return run_c3(args)
    if args.workload == "c5":
        return run_c5(args)
    if args.workload == "sigma":
        return run_sigma(args)
    if args.workload == "real":
        return run_real(args)
    if args.workload == "eps":
        return run_eps(args)
    if args.workload != "c2":
        raise SystemExit(f"bench.py: unknown workload {args.workload}")
    t0 = time.perf_counter()
    cr = crystal_for(args.workload)
    t_fix = time.perf_counter() - t0
    print(f"[bench] fixture {args.workload} built in {t_fix:.1f} s", file=sys.stderr, flush=True)
    ng, nw = cr.gmill.shape[0], len(cr.omegas)
    forms = {}
    ref_E = None
    for prec in args.forms.split(","):
        f, E = run_form(cr, prec, args.steps, args.warmup, ref_E)
        if prec == "fp64":
            ref_E = E
        forms[prec] = f
        print(f"[bench] {prec}: {f['ms_per_step']:.2f} ms/step (rho {f['t_rho_ms']:.2f}, chi0 "
              f"{f['t_chi0_ms']:.2f}, eps {f['t_eps_ms']:.2f}) e_F={f.get('e_F_vs_fp64')}", file=sys.stderr,
              flush=True)
    K = forms[next(iter(forms))]["K"]
    # the reported form is the split-bf16 one when it was timed and passes the gate; plain bf16
    # (no split correction) is timed beside it but never reported
    ok = [p for p in forms if p != "bf16" and (p == "fp64" or "fp64" not in forms
                                               or forms[p].get("e_F_vs_fp64", 1.0) <= GATE)]
    best = "bf16x3" if "bf16x3" in ok else min(ok, key=lambda p: forms[p]["ms_per_step"])
    fb = forms[best]
    t = fb["ms_per_step"] * 1e-3
    res = {
        "metric": "chi0 GFLOP/s + transitions/s per q,w; speedup vs FP64 at eps^-1 rel err<=1e-4",
        "value": chi0_flops(K, ng, nw) / t / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": fb["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[best],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: fcc 4x4x4 k, 16 occ + 200 empty bands, FFT 36^3, "
                               f"NG={ng}, {nw} imaginary frequencies, K={K} transitions",
                   "form": best, "global_batch": K, "parallelism": "single GPU"},
        "transitions_per_s_per_qw": K * nw / t,
        "speedup_vs_fp64": forms["fp64"]["ms_per_step"] / fb["ms_per_step"] if "fp64" in forms else None,
        "e_F_vs_fp64": fb.get("e_F_vs_fp64", 0.0),
        "stage_ms": {"rho": fb["t_rho_ms"], "chi0": fb["t_chi0_ms"], "eps": fb["t_eps_ms"]},
        "fp64_ms_per_step": forms.get("fp64", {}).get("ms_per_step"),
        "roofline": roofline(cr, fb, K, nw, ng),
        "fixture_s": t_fix,
    }
    # the oscillator-strength kernel of the same step, for reference
    rk = [k for k in fb["kernels"] if k.startswith("rho_gemm") or k in ("rho_yz", "rho_zy")]
    if rk and rk[0] != res["roofline"]["kernel"]:
        res["roofline_rho"] = roofline(cr, fb, K, nw, ng, name=rk[0])
    # the chi0 kernel of every form timed, against the MFMA peak of its own precision
    res["roofline_chi0_by_form"] = {
        p: roofline(cr, f, K, nw, ng, name=next(k for k in f["kernels"] if k.startswith("chi0_tiles")
                                                or k.startswith("chi0_blocks")))
        for p, f in forms.items()}
    if not args.no_cpu:
        print("[bench] timing the oracle on the host cores", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(cr, args.cpu_pairs)
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = 2 * a.numel() * 8
    if args.detail:
        with open(args.detail, "w") as fh:
            json.dump(dict(result=res, forms=forms), fh, indent=1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

"""Train the learned band tail on the GPU and evaluate it on held-out crystals.

    python -m paper_1902_03837_amd.train_tail --out tail_model.npz [--train 64 --test 16 --epochs 12]

Training data: chi0 of seeded crystals of the learned-tail workload (fcc, 4
k-points, q = X_z, 8 occupied bands, 59 G-vectors, 8 imaginary frequencies)
summed over 50, 100 and all 1000 empty bands by the plain FP64 path. Features
and targets come from xo_tail_features, the two ensemble members are trained
with the xo MLP kernels (Adam, MSE), and each held-out crystal is evaluated by the
relative error of eps~^-1 against the full band sum for (a) the truncated sum,
(b) the truncated sum plus the Bruneval-Gonze terminator (App. B, extrapolar
energy 1.5 Ha above the last explicit band) and (c) the truncated sum plus the
learned tail, with the time of each path. With --model the training is skipped
and the given model is evaluated.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import xo
from . import tail as T
from .pipeline import DeviceCrystal, qpg as qpg_of


def log(msg):
    print(msg, flush=True)


def rel_err(E, R):
    return max(float(torch.linalg.norm(E[j] - R[j]) / torch.linalg.norm(R[j])) for j in range(R.shape[0]))


def _train(args, train_seeds, ntrunc, nhalf):
    from synth import crystal_for
    assert args.out, "training needs --out"
    # ---- training crystals: chi0 over nhalf, ntrunc and all empty bands (FP64 path)
    geo, chis_all = [], []
    t0 = time.time()
    for i, s in enumerate(train_seeds):
        t1 = time.time()
        cr = crystal_for(args.workload, seed=s)
        t2 = time.time()
        chis, _ = T.crystal_tensors(cr, ntrunc, nhalf, base=args.base)
        torch.cuda.synchronize()
        geo.append((qpg_of(cr), T.gdiff_table(cr), cr.omegas, cr.gmill.shape[0]))
        chis_all.append(chis)
        log(f"[tail] train crystal {i + 1}/{len(train_seeds)} seed {s}: fixture {t2 - t1:.1f} s, "
            f"gpu {time.time() - t2:.2f} s")
        del cr
    ones, zeros = np.ones(T.NFEAT, np.float32), np.zeros(T.NFEAT, np.float32)

    def features(mu, isd, tsc):
        Xs, Ts = [], []
        for (qpg, gd, w, ng), chis in zip(geo, chis_all):
            n = len(w) * ng * ng
            X = torch.empty((n, T.NFEAT), dtype=torch.float32, device="cuda")
            Tt = torch.empty((n, 2), dtype=torch.float32, device="cuda")
            xo.tail_features(chis[1], chis[0], qpg, gd, w, mu, isd, X, chi_f=chis[2], T=Tt, tsc=tsc)
            Xs.append(X)
            Ts.append(Tt)
        return torch.cat(Xs), torch.cat(Ts)

    Xr, Tr = features(zeros, ones, 1.0)
    mu, isd, tsc = T.normalise(Xr, Tr)
    del Xr, Tr
    X, Tt = features(mu, isd, tsc)
    lo, hi = T.feature_range(X)
    log(f"[tail] training set: {X.shape[0]} samples, target scale {tsc:.3e}, built in {time.time() - t0:.1f} s")

    members, hists = [], []
    t3 = time.time()
    for ms in (1, 2):
        p, h = T.train(X, Tt, ms, args.epochs, args.batch, args.lr, log=log)
        members.append(p)
        hists.append(h)
    torch.cuda.synchronize()
    t_train = time.time() - t3
    model = T.TailModel(members, mu, isd, tsc, lo, hi, base=args.base)
    model.save(args.out)
    log(f"[tail] trained 2 members in {t_train:.1f} s -> {args.out}")
    del X, Tt, chis_all

    return model, t_train, hists, geo


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="where to save the trained model")
    ap.add_argument("--train", type=int, default=64)
    ap.add_argument("--test", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--report", default=None)
    ap.add_argument("--model", default=None, help="evaluate this trained model instead of training one")
    ap.add_argument("--base", default="bg", choices=("trunc", "bg"),
                    help="what the network corrects: the truncated sum or it plus the terminator")
    args = ap.parse_args(argv)
    from synth import crystal_for, CONFIGS
    spec = CONFIGS[args.workload]
    ntrunc = spec["ntrunc"]
    nhalf = ntrunc // 2
    seed0 = spec["seed"]
    train_seeds = list(range(seed0, seed0 + args.train))
    test_seeds = list(range(2 * seed0, 2 * seed0 + args.test))

    if args.model:
        model = T.TailModel.load(args.model)
        t_train, hists, geo = 0.0, [[float("nan")], [float("nan")]], None
        log(f"[tail] evaluating {args.model}")
    else:
        model, t_train, hists, geo = _train(args, train_seeds, ntrunc, nhalf)
    # ---- held-out evaluation
    rows = []
    for i, s in enumerate(test_seeds):
        cr = crystal_for(args.workload, seed=s)
        qpg = qpg_of(cr)
        dc = DeviceCrystal.upload(cr, "fp64")
        ng, nw = cr.gmill.shape[0], len(cr.omegas)
        E = {k: torch.empty((nw, ng, ng), dtype=torch.complex128, device="cuda")
             for k in ("full", "trunc", "learn", "bg")}
        nfull = cr.coef[0].shape[0] - cr.nocc
        # full band sum
        st = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ev[0].record(st)
        chi_f = T.chi0_blocks(dc, [nfull])[0]
        xo.epsinv(chi_f, qpg, out=E["full"])
        ev[1].record(st)
        # learned tail (guarded) on its base: the truncated sum, or it plus the terminator
        if model.base == "bg":
            chi_t0 = T.chi0_blocks(dc, [ntrunc])[0]
            chis = [chi_t0, T.xterm_chi0(dc, ntrunc, chi_t0)]
        else:
            chis = T.chi0_blocks(dc, [nhalf, ntrunc])
        chi_l, info = T.predict(model, cr, chis)
        used = "learned"
        if chi_l is None:
            used = "fallback"
            chi_l = T.chi0_blocks(dc, [nfull])[0]
        xo.epsinv(chi_l, qpg, out=E["learn"])
        ev[2].record(st)
        chi_trunc = chis[0] if model.base == "bg" else chis[1]
        xo.epsinv(chi_trunc, qpg, out=E["trunc"])
        ev[3].record(st)
        # truncated sum + Bruneval-Gonze terminator (its own rho and chi0 of the explicit bands)
        ev[4].record(st)
        chi_t = T.chi0_blocks(dc, [ntrunc])[0]
        chi_bg = T.xterm_chi0(dc, ntrunc, chi_t)
        xo.epsinv(chi_bg, qpg, out=E["bg"])
        ev[5].record(st)
        torch.cuda.synchronize()
        r = dict(seed=s, e_trunc=rel_err(E["trunc"], E["full"]), e_learned=rel_err(E["learn"], E["full"]),
                 e_bg=rel_err(E["bg"], E["full"]),
                 chi0_trunc_err=rel_err(chi_trunc, chi_f), chi0_learned_err=rel_err(chi_l, chi_f),
                 chi0_bg_err=rel_err(chi_bg, chi_f),
                 t_full_ms=ev[0].elapsed_time(ev[1]), t_learned_ms=ev[1].elapsed_time(ev[2]),
                 t_bg_ms=ev[4].elapsed_time(ev[5]), path=used, **info)
        rows.append(r)
        log(f"[tail] held-out {i + 1}/{len(test_seeds)} seed {s}: e_F trunc {r['e_trunc']:.3e} BG {r['e_bg']:.3e} "
            f"learned {r['e_learned']:.3e} ({used}); t full {r['t_full_ms']:.2f} ms BG {r['t_bg_ms']:.2f} ms "
            f"learned {r['t_learned_ms']:.2f} ms")
        del dc, cr
    summ = dict(workload=args.workload, train=len(train_seeds), test=len(test_seeds), epochs=args.epochs,
                model=args.model or args.out, base=model.base, t_train_s=t_train,
                final_loss=[h[-1] for h in hists],
                median_e_trunc=float(np.median([r["e_trunc"] for r in rows])),
                median_e_bg=float(np.median([r["e_bg"] for r in rows])),
                median_t_full_ms=float(np.median([r["t_full_ms"] for r in rows])),
                median_t_bg_ms=float(np.median([r["t_bg_ms"] for r in rows])),
                median_t_learned_ms=float(np.median([r["t_learned_ms"] for r in rows])),
                median_e_learned=float(np.median([r["e_learned"] for r in rows])),
                worst_e_learned=float(max(r["e_learned"] for r in rows)),
                fallbacks=sum(r["path"] == "fallback" for r in rows), rows=rows)
    log(json.dumps({k: v for k, v in summ.items() if k != "rows"}))
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(summ, fh, indent=1)


if __name__ == "__main__":
    main()

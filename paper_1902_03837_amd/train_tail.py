"""Train the learned band tail on the GPU and evaluate it on held-out crystals.

    python -m paper_1902_03837_amd.train_tail --out tail_model.npz [--workload c4 --train 64 --test 16]
    python -m paper_1902_03837_amd.train_tail --workload c5 --train 8 --test 2 --prec bf16x3 \\
        --samples 2000000 --out tail_model_c5.npz --report c5_report.json

Training data: chi0 of seeded crystals of the workload summed over the ntrunc lowest
empty bands, that sum plus the Bruneval-Gonze terminator (App. B, extrapolar energy
1.5 Ha above the last explicit band), and all empty bands, by the path in --prec.
Features and targets come from xo_tail_features; with --samples only that many
elements of each crystal (every diagonal element and a seeded uniform draw of the rest)
enter the training set, while the guard's feature range covers every element. The two
ensemble members are trained with the xo MLP kernels (Adam, MSE).

Each held-out crystal is judged against the plain FP64 full band sum (relative
Frobenius error of eps~^-1, worst frequency) for four paths run in --prec, each timed
from the orbitals to eps~^-1 with HIP events: the full band sum; the truncated sum; the
truncated sum plus the terminator; and that plus the learned remainder (the guard may
send a crystal to the full sum instead). With --model the training is skipped.
"""

from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import xo
from . import tail as T
from .pipeline import DeviceCrystal, chi0_pref, ntrans, qpg as qpg_of, rho_all, run_crystal


def log(msg):
    print(msg, flush=True)


def rel_err(E, R):
    return max(float(torch.linalg.norm(E[j] - R[j]) / torch.linalg.norm(R[j])) for j in range(R.shape[0]))


def _crystal(workload, seed, cache):
    from synth import crystal_for
    progress = lambda m: log(f"[tail]   fixture seed {seed}: {m}")  # noqa: E731
    if cache:
        from synth.cache import cached_crystal
        return cached_crystal(workload, cache, seed=seed, progress=progress)
    return crystal_for(workload, seed=seed, progress=progress)


def _sample_rows(n, ng, nw, count, seed, dev):
    """Every diagonal element and a seeded uniform draw of the others (row indices of
    [nw][ng][ng], duplicates dropped). The diagonal, whose large elements carry a quarter to
    a half of the terminator's residual, is always in; a purely uniform draw of twice the size
    judged no better on the large cell (e_F 1.69e-2 against 1.64e-2 on the first held-out
    crystal)."""
    g = np.random.default_rng(seed)
    diag = (np.arange(nw)[:, None] * ng * ng + np.arange(ng)[None, :] * (ng + 1)).reshape(-1)
    rest = g.integers(0, n, max(0, count - diag.size))
    return torch.from_numpy(np.unique(np.concatenate([diag, rest])).astype(np.int32)).to(dev)


def _train(args, train_seeds, ntrunc, nhalf):
    assert args.out, "training needs --out"
    dev = "cuda"
    ones, zeros = np.ones(T.NFEAT, np.float32), np.zeros(T.NFEAT, np.float32)
    geo, chis_all, rows = [], [], []
    t0 = time.time()
    for i, s in enumerate(train_seeds):
        t1 = time.time()
        cr = _crystal(args.workload, s, args.fixture_cache)
        t2 = time.time()
        chis, _ = T.crystal_tensors(cr, ntrunc, nhalf, base=args.base, prec=args.prec, shift=args.shift)
        torch.cuda.synchronize()
        ng, nw = cr.gmill.shape[0], len(cr.omegas)
        n = nw * ng * ng
        geo.append((qpg_of(cr), cr.gmill, cr.lat.bvec, cr.omegas, ng))
        chis_all.append(chis)
        rows.append(_sample_rows(n, ng, nw, args.samples, s, dev) if args.samples else None)
        log(f"[tail] train crystal {i + 1}/{len(train_seeds)} seed {s}: fixture {t2 - t1:.1f} s, "
            f"gpu {time.time() - t2:.2f} s" + (f", {rows[-1].numel()} of {n} elements" if args.samples else ""))
        del cr
        torch.cuda.empty_cache()

    def features(mu, isd, tsc, want_range=False):
        """Training rows of every crystal (all elements, or the sampled ones); with want_range
        also the min and max of every feature over all elements."""
        Xs, Ts = [], []
        lo, hi = np.full(T.NFEAT, np.inf, np.float32), np.full(T.NFEAT, -np.inf, np.float32)
        for (qpg, gm, bv, w, ng), chis, idx in zip(geo, chis_all, rows):
            n = len(w) * ng * ng
            X = torch.empty((n, T.NFEAT), dtype=torch.float32, device=dev)
            Tt = torch.empty((n, 2), dtype=torch.float32, device=dev)
            xo.tail_features(chis[1], chis[0], qpg, gm, bv, w, mu, isd, X, chi_f=chis[2], T=Tt, tsc=tsc)
            if want_range:
                a, b = T.feature_range(X)
                lo, hi = np.minimum(lo, a), np.maximum(hi, b)
            if idx is not None:
                Xg = torch.empty((idx.numel(), T.NFEAT), dtype=torch.float32, device=dev)
                Tg = torch.empty((idx.numel(), 2), dtype=torch.float32, device=dev)
                xo.gather_rows(X, idx, Xg)
                xo.gather_rows(Tt, idx, Tg)
                X, Tt = Xg, Tg
            Xs.append(X)
            Ts.append(Tt)
        return torch.cat(Xs), torch.cat(Ts), lo, hi

    Xr, Tr, _, _ = features(zeros, ones, 1.0)
    mu, isd, tsc = T.normalise(Xr, Tr)
    del Xr, Tr
    X, Tt, lo, hi = features(mu, isd, tsc, want_range=True)
    del chis_all
    torch.cuda.empty_cache()
    log(f"[tail] training set: {X.shape[0]} samples, target scale {tsc:.3e}, built in {time.time() - t0:.1f} s")

    members, hists = [], []
    t3 = time.time()
    for ms in (1, 2):
        p, h = T.train(X, Tt, ms, args.epochs, args.batch, args.lr, log=log)
        members.append(p)
        hists.append(h)
    torch.cuda.synchronize()
    t_train = time.time() - t3
    model = T.TailModel(members, mu, isd, tsc, lo, hi, base=args.base, shift=args.shift)
    model.save(args.out)
    log(f"[tail] trained 2 members in {t_train:.1f} s -> {args.out}")
    return model, t_train, hists, int(X.shape[0])


class _Timer:
    def __init__(self):
        self.st = torch.cuda.current_stream()
        self.ev = []

    def mark(self):
        e = torch.cuda.Event(enable_timing=True)
        e.record(self.st)
        self.ev.append(e)

    def ms(self, i, j):
        return self.ev[i].elapsed_time(self.ev[j])


def _trunc_chi(dc, nempty):
    cr = dc.cr
    K, ng, nw = ntrans(cr, nempty), cr.gmill.shape[0], len(cr.omegas)
    M = torch.empty((K, ng), dtype=torch.complex128 if dc.prec == "fp64" else torch.complex64, device="cuda")
    dE = torch.empty(K, dtype=torch.float64, device="cuda")
    chi = torch.empty((nw, ng, ng), dtype=torch.complex128, device="cuda")
    rho_all(dc, M, dE, nempty)
    xo.chi0(M, dE, cr.omegas, chi0_pref(cr), out=chi, prec=dc.prec, check_dE=False)
    return chi


def evaluate(model, cr, ntrunc, prec):
    """The four paths of one held-out crystal, judged against the FP64 full band sum."""
    q = qpg_of(cr)
    ng, nw = cr.gmill.shape[0], len(cr.omegas)
    # judge: the plain FP64 path over every band
    dc64 = DeviceCrystal.upload(cr, "fp64")
    _, _, chi_ref, E_ref = run_crystal(dc64, check_dE=False)
    torch.cuda.synchronize()
    del dc64
    torch.cuda.empty_cache()
    dc = DeviceCrystal.upload(cr, prec)
    E = {k: torch.empty((nw, ng, ng), dtype=torch.complex128, device="cuda") for k in ("trunc", "bg", "learn")}
    run_crystal(dc, check_dE=False)          # warm-up: the path's tables, plans and workspaces
    torch.cuda.synchronize()
    tm = _Timer()
    tm.mark()
    _, _, chi_full, E_full = run_crystal(dc, check_dE=False)
    tm.mark()
    chi = _trunc_chi(dc, ntrunc)
    xo.epsinv(chi, q, out=E["trunc"])
    tm.mark()
    chi = _trunc_chi(dc, ntrunc)
    chi_bg = T.xterm_chi0(dc, ntrunc, chi, shift=model.shift)
    xo.epsinv(chi_bg, q, out=E["bg"])
    tm.mark()
    if model.base == "bg":    # the network corrects the terminator-corrected sum
        chi = _trunc_chi(dc, ntrunc)
        chis_in = [chi, T.xterm_chi0(dc, ntrunc, chi, shift=model.shift)]
    else:                     # it corrects the truncated sum; the slope is its upper half
        chis_in = T.chi0_blocks(dc, [ntrunc // 2, ntrunc], prec)
    tm.mark()
    chi_l, info = T.predict(model, cr, chis_in)   # reads the guard sums back (synchronises)
    tm.mark()
    used = "learned"
    if chi_l is None:
        used = "fallback"
        _, _, chi_l, E["learn"] = run_crystal(dc, check_dE=False)
    else:
        xo.epsinv(chi_l, q, out=E["learn"])
    tm.mark()
    torch.cuda.synchronize()
    r = dict(e_full=rel_err(E_full, E_ref), e_trunc=rel_err(E["trunc"], E_ref), e_bg=rel_err(E["bg"], E_ref),
             e_learned=rel_err(E["learn"], E_ref), chi0_learned_err=rel_err(chi_l, chi_ref),
             chi0_bg_err=rel_err(chi_bg, chi_ref), t_full_ms=tm.ms(0, 1), t_trunc_ms=tm.ms(1, 2),
             t_bg_ms=tm.ms(2, 3), t_learned_ms=tm.ms(3, 6), t_predict_ms=tm.ms(4, 5), path=used, **info)
    return r


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="where to save the trained model")
    ap.add_argument("--train", type=int, default=64)
    ap.add_argument("--test", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--ntrunc", type=int, default=None, help="explicit empty bands (default: the workload's)")
    ap.add_argument("--prec", default="fp64", choices=("fp64", "fp32", "bf16x3"),
                    help="precision of the chi0 paths (training data and the timed paths)")
    ap.add_argument("--samples", type=int, default=0, help="training elements per crystal (0: all)")
    ap.add_argument("--train-seed", type=int, default=None, help="first training seed (default: the workload's)")
    ap.add_argument("--test-seed", type=int, default=None, help="first held-out seed (default: twice that)")
    ap.add_argument("--fixture-cache", default=None, help="directory to keep generated crystals in (npz)")
    ap.add_argument("--report", default=None)
    ap.add_argument("--model", default=None, help="evaluate this trained model instead of training one")
    ap.add_argument("--base", default="bg", choices=("trunc", "bg"),
                    help="what the network corrects: the truncated sum or it plus the terminator")
    ap.add_argument("--shift", type=float, default=1.5,
                    help="terminator: extrapolar energy above the last explicit band (Ha)")
    args = ap.parse_args(argv)
    from synth import CONFIGS
    spec = CONFIGS[args.workload]
    ntrunc = args.ntrunc or spec["ntrunc"]
    nhalf = ntrunc // 2
    seed0 = spec["seed"] if args.train_seed is None else args.train_seed
    tseed0 = 2 * spec["seed"] if args.test_seed is None else args.test_seed
    train_seeds = list(range(seed0, seed0 + args.train))
    test_seeds = list(range(tseed0, tseed0 + args.test))
    assert not set(train_seeds) & set(test_seeds), "held-out seeds overlap the training seeds"
    xo.lib()

    if args.model:
        model = T.TailModel.load(args.model)
        t_train, hists, nsamp = 0.0, [[float("nan")], [float("nan")]], 0
        log(f"[tail] evaluating {args.model}")
    else:
        model, t_train, hists, nsamp = _train(args, train_seeds, ntrunc, nhalf)
    rows = []
    for i, s in enumerate(test_seeds):
        t0 = time.time()
        cr = _crystal(args.workload, s, args.fixture_cache)
        log(f"[tail] held-out {i + 1}/{len(test_seeds)} seed {s}: fixture {time.time() - t0:.1f} s")
        r = dict(seed=s, **evaluate(model, cr, ntrunc, args.prec))
        rows.append(r)
        log(f"[tail]   e_F vs FP64 full: full({args.prec}) {r['e_full']:.3e} trunc {r['e_trunc']:.3e} "
            f"BG {r['e_bg']:.3e} learned {r['e_learned']:.3e} ({r['path']}); ms: full {r['t_full_ms']:.1f} "
            f"trunc {r['t_trunc_ms']:.1f} BG {r['t_bg_ms']:.1f} learned {r['t_learned_ms']:.1f} "
            f"(predict {r['t_predict_ms']:.1f})")
        del cr
        torch.cuda.empty_cache()
    med = lambda k: float(np.median([r[k] for r in rows]))  # noqa: E731
    summ = dict(workload=args.workload, prec=args.prec, ntrunc=ntrunc, train=len(train_seeds),
                train_seeds=[train_seeds[0], train_seeds[-1]], test_seeds=test_seeds, samples_per_crystal=args.samples,
                training_samples=nsamp, epochs=args.epochs, batch=args.batch, model=args.model or args.out,
                base=model.base, shift=model.shift, t_train_s=t_train, final_loss=[h[-1] for h in hists],
                median_e_full=med("e_full"), median_e_trunc=med("e_trunc"), median_e_bg=med("e_bg"),
                median_e_learned=med("e_learned"), worst_e_learned=float(max(r["e_learned"] for r in rows)),
                median_t_full_ms=med("t_full_ms"), median_t_trunc_ms=med("t_trunc_ms"), median_t_bg_ms=med("t_bg_ms"),
                median_t_learned_ms=med("t_learned_ms"), median_t_predict_ms=med("t_predict_ms"),
                fallbacks=sum(r["path"] == "fallback" for r in rows), rows=rows)
    log(json.dumps({k: v for k, v in summ.items() if k != "rows"}))
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(summ, fh, indent=1)


if __name__ == "__main__":
    main()

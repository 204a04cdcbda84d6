"""Learned empty-band tail of chi0, trained and evaluated on the GPU.

The sum over empty states in Eq. (X_IP) converges slowly with the number of
bands; the paper corrects it with the extrapolar X-terminator (Eq. X_term_def,
Appendix B). Here an ensemble of two small MLPs predicts the missing tail
s_G (chi0_full - chi0_trunc) s_G' element by element from features of the
truncated sum (xo_tail_features). Guard: features outside the training range
(widened by 10 %) or an ensemble disagreement above tau send the crystal to the
full band sum, which is also the reference for the network's error.

Every arithmetic step runs in libxo kernels (rho, chi0, features, MLP forward,
backward, MSE, Adam, apply, guard); this module allocates device buffers,
draws the seeded minibatch permutations and sequences the calls.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import xo
from .pipeline import DeviceCrystal, band_ranges, chi0_pref, qpg

DIMS = [9, 256, 256, 256, 2]   # 3 hidden layers of 256, SiLU
NFEAT = 9


def chi0_blocks(dc: DeviceCrystal, cuts: List[int], prec: str = "fp64", stream=None):
    """chi0 summed over empty bands [0, cuts[0]), [0, cuts[1]), ... (cumulative).

    One batched rho call covers every (pair, band block); each block's rows sit
    contiguously in M so chi0 of the next block is an accumulate on a copy.
    """
    cr = dc.cr
    ng, nw = cr.gmill.shape[0], len(cr.omegas)
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    blocks = []
    lo = 0
    for hi in cuts:
        calls, off = [], 0
        for ik, ikp, g0, c_lo, c_hi, nv in band_ranges(cr):
            a, b = c_lo + lo, min(c_lo + hi, c_hi)
            if b <= a:
                continue
            calls.append((ik, ikp, g0, a, b, nv, off))
            off += (b - a) * nv
        blocks.append((calls, off))
        lo = hi
    total = sum(o for _, o in blocks)
    dev = dc.coef[0].device
    M = torch.empty((total, ng), dtype=cdt, device=dev)
    dE = torch.empty(total, dtype=torch.float64, device=dev)
    args, base, spans = [], 0, []
    for calls, n in blocks:
        for ik, ikp, g0, a, b, nv, off in calls:
            nc = b - a
            o = base + off
            args.append(dict(coef_c=dc.coef[ik][a:b], mill_c=cr.mill[ik], e_c=dc.eps[ik][a:b],
                             coef_v=dc.coef[ikp][:nv], mill_v=cr.mill[ikp], e_v=dc.eps[ikp][:nv],
                             gmill=cr.gmill, g0=g0, grid=cr.grid, out=M[o:o + nc * nv].view(nv, nc, ng),
                             dE=dE[o:o + nc * nv], prec=prec, kcart=cr.kcart(ik), bvec=cr.lat.bvec))
        spans.append((base, base + n))
        base += n
    xo.rho_batch(args, stream=stream)
    out = []
    chi = torch.empty((nw, ng, ng), dtype=torch.complex128, device=dev)
    for i, (a, b) in enumerate(spans):
        if i > 0:
            chi = chi.clone()
        xo.chi0(M[a:b], dE[a:b], cr.omegas, chi0_pref(cr), out=chi, prec=prec, accumulate=i > 0, check_dE=False,
                stream=stream)
        out.append(chi)
    return out


def xterm_chi0(dc: DeviceCrystal, nempty: int, chi_trunc, shift: float = 1.5, stream=None):
    """chi0 with the Bruneval-Gonze terminator (App. B): chi_trunc, summed over the
    nempty lowest empty bands, plus the correction of every k-pair (xo_rho over the
    explicit bands at k, occupied included, then xo_xterm), in the crystal's precision;
    ebar = highest explicit band energy at k + shift."""
    cr = dc.cr
    assert not cr.q0
    ng = cr.gmill.shape[0]
    cdt = torch.complex128 if dc.prec == "fp64" else torch.complex64
    out = chi_trunc.clone()
    for ik, ikp, g0, _, _, nv in band_ranges(cr):
        nb = cr.nocc_at(ik) + nempty
        M = torch.empty((nv * nb, ng), dtype=cdt, device=out.device)
        xo.rho(dc.coef[ik][:nb], cr.mill[ik], dc.eps[ik][:nb], dc.coef[ikp][:nv], cr.mill[ikp], dc.eps[ikp][:nv],
               cr.gmill, g0, cr.grid, out=M.view(nv, nb, ng), prec=dc.prec, kcart=cr.kcart(ik), bvec=cr.lat.bvec,
               stream=stream)
        ebar = float(cr.eps[ik][nb - 1]) + shift
        xo.xterm(dc.coef[ikp][:nv], cr.mill[ikp], dc.eps[ikp][:nv], ebar, cr.gmill, cr.omegas, chi0_pref(cr), M, nb, out,
                 prec=dc.prec, stream=stream)
    return out


class MLP:
    """Device-resident MLP parameters with Adam state."""

    def __init__(self, params_flat: np.ndarray, dims=DIMS, device="cuda"):
        self.dims = list(dims)
        self.p = torch.from_numpy(np.ascontiguousarray(params_flat, np.float32)).to(device)
        self.g = torch.zeros_like(self.p)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.step = 0
        self._ws = {}

    def _bufs(self, n):
        if n not in self._ws:
            dev = self.p.device
            na = sum(2 * n * w for w in self.dims[1:-1])
            wmax = max(self.dims)
            self._ws[n] = (torch.empty(na, dtype=torch.float32, device=dev),
                           torch.empty((n, self.dims[-1]), dtype=torch.float32, device=dev),
                           torch.empty(2 * n * wmax, dtype=torch.float32, device=dev))
        return self._ws[n]

    def forward(self, X, n=None):
        n = X.shape[0] if n is None else n
        acts, Y, _ = self._bufs(n)
        xo.mlp_forward(self.dims, self.p, X, n, acts, Y)
        return Y

    def backward(self, X, dY, dX=None):
        n = X.shape[0]
        acts, _, work = self._bufs(n)
        xo.mlp_backward(self.dims, self.p, X, n, acts, dY, self.g, work, dX)
        return self.g

    def adam(self, lr):
        self.step += 1
        xo.adam_step(self.p, self.g, self.m, self.v, lr, self.step)


@dataclass
class TailModel:
    members: List[np.ndarray]       # flat FP32 parameters of each ensemble member
    mu: np.ndarray
    isd: np.ndarray
    tsc: float
    lo: np.ndarray                  # normalised feature range seen in training
    hi: np.ndarray
    tau: float = 0.25
    dims: List[int] = field(default_factory=lambda: list(DIMS))
    base: str = "trunc"             # what the network corrects: the truncated sum, or it plus the terminator
    shift: float = 1.5              # terminator: extrapolar energy above the last explicit band (Ha)
    info: dict = field(default_factory=dict)

    def save(self, path):
        np.savez(path, members=np.stack(self.members), mu=self.mu, isd=self.isd, tsc=self.tsc, lo=self.lo,
                 hi=self.hi, tau=self.tau, dims=np.array(self.dims), base=np.array(self.base), shift=self.shift)

    @classmethod
    def load(cls, path):
        z = np.load(path, allow_pickle=False)
        base = str(z["base"]) if "base" in z.files else "trunc"
        shift = float(z["shift"]) if "shift" in z.files else 1.5
        return cls(list(z["members"]), z["mu"], z["isd"], float(z["tsc"]), z["lo"], z["hi"], float(z["tau"]),
                   [int(x) for x in z["dims"]], base, shift)


def crystal_tensors(cr, ntrunc, nhalf, with_full=True, prec="fp64", base="trunc", shift=1.5):
    """[reference, base, (full)] chi0 of one crystal on the device.

    base "trunc": [sum over nhalf, sum over ntrunc, full sum] (the network corrects
    the truncated sum; the slope feature is the last block of bands).
    base "bg": [sum over ntrunc, that plus the Bruneval-Gonze terminator, full sum]
    (the network corrects the terminator, extrapolar energy `shift` above the last explicit
    band; the slope feature is the terminator's own correction)."""
    dc = DeviceCrystal.upload(cr, prec)
    full = [cr.coef[0].shape[0] - cr.nocc] if with_full else []
    if base == "trunc":
        return chi0_blocks(dc, [nhalf, ntrunc] + full, prec), dc
    assert base == "bg"
    chis = chi0_blocks(dc, [ntrunc] + full, prec)
    return [chis[0], xterm_chi0(dc, ntrunc, chis[0], shift=shift)] + chis[1:], dc


def build_features(cr, chis, mu, isd, tsc, dev="cuda"):
    ng, nw = cr.gmill.shape[0], len(cr.omegas)
    n = nw * ng * ng
    X = torch.empty((n, NFEAT), dtype=torch.float32, device=dev)
    T = torch.empty((n, 2), dtype=torch.float32, device=dev) if len(chis) > 2 else None
    xo.tail_features(chis[1], chis[0], qpg(cr), cr.gmill, cr.lat.bvec, cr.omegas, mu, isd, X,
                     chi_f=chis[2] if len(chis) > 2 else None, T=T, tsc=tsc)
    return X, T


def make_training_set(crystals_fn, seeds, ntrunc, nhalf, log=print):
    """Raw (unnormalised) features and targets of every training crystal, on the device."""
    Xs, Ts = [], []
    one = np.ones(NFEAT, np.float32)
    zero = np.zeros(NFEAT, np.float32)
    for i, s in enumerate(seeds):
        t0 = time.time()
        cr = crystals_fn(s)
        t1 = time.time()
        chis, _ = crystal_tensors(cr, ntrunc, nhalf)
        X, T = build_features(cr, chis, zero, one, 1.0)
        Xs.append(X)
        Ts.append(T)
        torch.cuda.synchronize()
        log(f"[tail] crystal {i + 1}/{len(seeds)} seed {s}: fixture {t1 - t0:.1f}s, gpu {time.time() - t1:.2f}s")
    return torch.cat(Xs), torch.cat(Ts)


def normalise(X, T):
    """mu, isd per feature and the target scale, from xo_col_stats; applied in place."""
    st = torch.empty((NFEAT, 4), dtype=torch.float64, device=X.device)
    xo.col_stats(X, st)
    s = st.cpu().numpy()
    mu = s[:, 0].astype(np.float32)
    sd = s[:, 1]
    isd = np.where(sd > 1e-12, 1.0 / np.maximum(sd, 1e-12), 1.0).astype(np.float32)
    st2 = torch.empty((2, 4), dtype=torch.float64, device=X.device)
    xo.col_stats(T, st2)
    tsd = float(max(st2.cpu().numpy()[:, 1].max(), 1e-30))
    return mu, isd, 1.0 / tsd


def train(X, T, seed, epochs, batch=4096, lr=1e-3, log=print, dims=DIMS):
    """Adam on MSE with xo kernels; minibatch order from a seeded permutation."""
    from synth.rand import mlp_init, flatten_params
    dev = X.device
    n = X.shape[0]
    net = MLP(flatten_params(mlp_init(dims, seed)), dims, dev)
    xb = torch.empty((batch, X.shape[1]), dtype=torch.float32, device=dev)
    tb = torch.empty((batch, T.shape[1]), dtype=torch.float32, device=dev)
    dY = torch.empty_like(tb)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    part = torch.empty(256, dtype=torch.float32, device=dev)
    g = np.random.default_rng(seed)
    nb = n // batch
    total = epochs * nb
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(g.permutation(n)[: nb * batch].astype(np.int32)).to(dev)
        acc = 0.0
        for b in range(nb):
            it = ep * nb + b
            lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * it / total))
            idx = perm[b * batch:(b + 1) * batch]
            xo.gather_rows(X, idx, xb)
            xo.gather_rows(T, idx, tb)
            Y = net.forward(xb)
            xo.mse(Y, tb, dY, loss, part)
            net.backward(xb, dY)
            net.adam(lr_t)
            if b % 64 == 0:
                acc = float(loss.item())
        hist.append(acc)
        log(f"[tail] member seed {seed} epoch {ep + 1}/{epochs} minibatch loss {acc:.4e}")
    return net.p.cpu().numpy(), hist


def feature_range(X):
    st = torch.empty((X.shape[1], 4), dtype=torch.float64, device=X.device)
    xo.col_stats(X, st)
    s = st.cpu().numpy()
    return s[:, 2].astype(np.float32), s[:, 3].astype(np.float32)


def predict(model: TailModel, cr, chis_trunc, dev="cuda", stream=None):
    """chi0 = chi0_trunc + learned tail, or None if the guard asks for the full sum.

    chis_trunc = [chi_ref, chi_base] (the slope reference and the sum the network corrects).
    One fused launch (xo_tail_predict) forms the features, runs both ensemble members on the
    matrix cores and sums the guard statistics; xo_tail_apply adds the tail. Returns (chi, stats)."""
    ng, nw = cr.gmill.shape[0], len(cr.omegas)
    Y = torch.empty((nw * ng * ng, 2), dtype=torch.float32, device=dev)
    stats = torch.empty(3, dtype=torch.float64, device=dev)
    params = torch.from_numpy(np.ascontiguousarray(np.stack(model.members), np.float32)).to(dev)
    q = qpg(cr)
    xo.tail_predict(chis_trunc[1], chis_trunc[0], q, cr.gmill, cr.lat.bvec, cr.omegas, model.mu, model.isd,
                    model.lo, model.hi, model.dims, params, Y, stats, stream=stream)
    st = stats.cpu().numpy()
    dis = float(np.sqrt(st[1] / max(st[2], 1e-300)))
    info = dict(out_of_range=int(st[0]), disagreement=dis)
    if st[0] > 0 or dis > model.tau:
        return None, info
    out = torch.empty_like(chis_trunc[1])
    xo.tail_apply(chis_trunc[1], Y, q, model.tsc, out, stream=stream)
    return out, info

"""Whole-crystal oracle: all k-pairs -> M, Delta -> chi0 -> eps~^-1. TEST INFRASTRUCTURE (oracle).

Transitions are ordered pair by pair (the crystal's k-pair list), and within a
pair as t = v * nc + c. Delta_t = e_{c,k} - e_{v,k'} (Eq. X_IP pole energy).
At q = 0 the G = 0 column is replaced by the velocity form of the head
(Eq. dip) along qhat, and the G != 0 columns use k' = k, G0 = 0.
"""

from __future__ import annotations

import numpy as np

from .rho import rho_direct, rho_fft, rho_head_q0
from .chi0 import chi0_from_rho, crystal_prefactor
from .epsinv import epsinv_sym, crystal_qpg


def rho_pair(cr, ipair, route="fft", nempty=None, band_lo=None, qhat=(1.0, 0.0, 0.0)):
    ik, ikp, g0 = cr.pairs[ipair]
    lo = cr.nocc_at(ik) if band_lo is None else band_lo
    hi = cr.coef[ik].shape[0] if nempty is None else cr.nocc_at(ik) + nempty
    nv = cr.nocc_at(ikp)
    cc, mc, ec = cr.coef[ik][lo:hi], cr.mill[ik], cr.eps[ik][lo:hi]
    cv, mv, ev = cr.coef[ikp][:nv], cr.mill[ikp], cr.eps[ikp][:nv]
    if route == "fft":
        r = rho_fft(cc, mc, cv, mv, cr.gmill, g0, cr.grid)
    else:
        r = rho_direct(cc, mc, cv, mv, cr.gmill, g0)
    if cr.q0:
        qh = np.asarray(qhat, float)
        qh = qh / np.linalg.norm(qh)
        i0 = int(np.nonzero(np.all(cr.gmill == 0, axis=1))[0][0])
        r[:, :, i0] = rho_head_q0(cc, ec, cv, ev, mc, cr.kcart(ik), cr.lat.bvec, qh)
    dE = ec[None, :] - ev[:, None]
    return r.reshape(-1, r.shape[-1]), dE.reshape(-1)


def rho_all_pairs(cr, route="fft", nempty=None, band_lo=None):
    Ms, dEs = [], []
    for ip in range(len(cr.pairs)):
        m, d = rho_pair(cr, ip, route, nempty, band_lo)
        Ms.append(m)
        dEs.append(d)
    return np.concatenate(Ms), np.concatenate(dEs)


def chi0_crystal(cr, route="fft", nempty=None):
    M, dE = rho_all_pairs(cr, route, nempty)
    return chi0_from_rho(M, dE, cr.omegas, crystal_prefactor(cr))


def epsinv_crystal(cr, route="fft", nempty=None):
    chi = chi0_crystal(cr, route, nempty)
    return epsinv_sym(chi, crystal_qpg(cr)), chi

"""Bruneval-Gonze extrapolar correction of chi0 (X-terminator). TEST INFRASTRUCTURE (oracle).

X-terminator subsection (Eq. X_term_def) and Appendix B (Eqs. rhotw-term,
F-term, X-term): the empty states above the last explicit band N_b' are given
one common extrapolar energy ebar, so their sum collapses by closure over the
complete set of states at k:

    sum_{c > N_b'} rho_cv(G) conj(rho_cv(G'))
        = <v| e^{-i(q+G').r} e^{i(q+G).r} |v>  -  sum_{n <= N_b'} rho_nv(G) conj(rho_nv(G'))
        = <v| e^{i(G-G').r} |v>               -  sum_{n <= N_b'} rho_nv(G) conj(rho_nv(G')),

where n runs over every explicit band at k, occupied ones included. At
imaginary frequency, with the sign of Eq. (X_IP) as read for the plain sum,

    Delta chi_GG'(q, i w) = -pref sum_{k, v} W(w, ebar_k - e_v)
                              [ <v| e^{i(G-G').r} |v> - sum_{n <= N_b'} rho_nv(G) conj(rho_nv(G')) ],
    W(w, D) = 2 D / (w^2 + D^2),  ebar_k = e_{N_b', k} + 1.5 Ha (the paper's default shift).

Readings: the printed density element <m|e^{i(G'+G).r}|m> is taken with the
difference G - G' that the closure of rho(G) rho*(G') produces, and the
subtracted term R of Eq. (X-term) is taken without occupation factors over all
explicit bands (the closure removes occupied states as well). The q -> 0 head
is not treated (the correction is applied at q != 0).
"""

from __future__ import annotations

import numpy as np

from .rho import rho_direct
from .chi0 import pole_weights, crystal_prefactor


def density_elements(coef, mill, kmill):
    """<v| e^{iK.r} |v> for every band v of one k and every Miller vector K: [nv][nK].

    With psi_v = e^{ik.r} sum_G c_v(G) e^{iG.r} the cell average picks
    sum_G conj(c_v(G + K)) c_v(G); this is rho_direct with the band on both sides.
    """
    nv = coef.shape[0]
    full = rho_direct(coef, mill, coef, mill, np.asarray(kmill, dtype=np.int64), np.zeros(3, dtype=np.int64))
    return full[np.arange(nv), np.arange(nv), :]


def xterm_bg(cr, nempty_explicit: int, shift: float = 1.5, rho_route=None):
    """Delta chi [nw][NG][NG] for the truncated sum over nempty_explicit empty bands."""
    assert not cr.q0, "the terminator is applied at q != 0"
    G = cr.gmill.astype(np.int64)
    ng, nw = G.shape[0], len(cr.omegas)
    diff = (G[:, None, :] - G[None, :, :]).reshape(-1, 3)
    kuniq, kidx = np.unique(diff, axis=0, return_inverse=True)
    kidx = kidx.reshape(ng, ng)
    out = np.zeros((nw, ng, ng), dtype=np.complex128)
    pref = crystal_prefactor(cr)
    for ik, ikp, g0 in cr.pairs:
        nb = cr.nocc_at(ik) + nempty_explicit          # explicit bands n <= N_b' at k
        ebar = cr.eps[ik][nb - 1] + shift
        nv = cr.nocc_at(ikp)
        cv, mv, ev = cr.coef[ikp][:nv], cr.mill[ikp], cr.eps[ikp][:nv]
        D = density_elements(cv, mv, kuniq)[:, kidx]   # [nv][G][G'] = <v|e^{i(G-G').r}|v>
        R = (rho_route or rho_direct)(cr.coef[ik][:nb], cr.mill[ik], cv, mv, G, np.asarray(g0))  # [nv][n][G]
        S = np.einsum("vng,vnh->vgh", R, np.conj(R))
        for j, w in enumerate(cr.omegas):
            wt = pole_weights(ebar - ev, w)
            out[j] += -pref * np.einsum("v,vgh->gh", wt, D - S)
    return out

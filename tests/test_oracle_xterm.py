"""Pins of the X-terminator oracle (Appendix B), CPU only."""

from dataclasses import replace

import numpy as np

from synth.crystal import fcc_lattice, make_crystal, shell_potential, ecut_for_npw
from synth.configs import A_FCC, FCC4
from oracle.pipeline import chi0_crystal
from oracle.terminator import xterm_bg, density_elements


def _free_crystal(npw=400):
    lat = fcc_lattice(A_FCC)
    return make_crystal(lat, shell_potential(lat, 0, zero=True), FCC4, np.array([.5, .5, 0.]), (20,) * 3,
                        ecut_for_npw(lat, npw), 9, None, 15, 3, 21, scissor_min=None, nocc_k=[9, 6, 6, 6])


def test_terminator_exact_when_upper_bands_sit_at_the_extrapolar_energy():
    """Free electrons in a complete finite basis whose k-spheres contain every e^{i(q+G).r}|v>:
    if every band above N_b' has exactly the energy ebar, the terminator is the exact
    remainder of the sum (the closure over all bands at k is exact)."""
    cr = _free_crystal()
    nbp, shift = 6, 1.5
    eps_mod = []
    for ik in range(len(cr.kf)):
        e = cr.eps[ik].copy()
        nb = cr.nocc_at(ik) + nbp
        e[nb:] = e[nb - 1] + shift
        eps_mod.append(e)
    cr_mod = replace(cr, eps=eps_mod)
    full = chi0_crystal(cr_mod)
    trunc = chi0_crystal(cr, nempty=nbp)
    dchi = xterm_bg(cr, nbp, shift)
    assert np.abs(trunc + dchi - full).max() < 1e-12 * np.abs(full).max()
    # and the correction is not negligible: without it the truncated sum is off
    assert np.abs(trunc - full).max() > 1e-2 * np.abs(full).max()


def test_terminator_with_the_printed_sum_g_plus_gprime_is_not_exact():
    """The printed <m|e^{i(G'+G).r}|m> breaks the identity above; the difference G - G' keeps it."""
    cr = _free_crystal()
    G = cr.gmill.astype(np.int64)
    ik, ikp, _ = cr.pairs[0]
    nv = cr.nocc_at(ikp)
    cv, mv = cr.coef[ikp][:nv], cr.mill[ikp]
    dsum = density_elements(cv, mv, (G[:, None, :] + G[None, :, :]).reshape(-1, 3)).reshape(nv, len(G), len(G))
    ddif = density_elements(cv, mv, (G[:, None, :] - G[None, :, :]).reshape(-1, 3)).reshape(nv, len(G), len(G))
    assert np.allclose(np.diagonal(ddif, axis1=1, axis2=2), 1.0)      # <v|v> = 1 on the diagonal
    assert np.abs(dsum - ddif).max() > 0.5


def test_terminator_is_hermitian_and_vanishes_with_no_gap_to_fill():
    cr = _free_crystal(npw=250)
    d = xterm_bg(cr, 4)
    for j in range(d.shape[0]):
        assert np.allclose(d[j], d[j].conj().T, atol=1e-14)
    # all bands explicit: nothing is left above N_b', the closure term equals the explicit sum
    nmax = min(cr.coef[ik].shape[0] - cr.nocc_at(ik) for ik in range(len(cr.kf)))
    full = xterm_bg(cr, nmax)
    assert np.abs(full).max() < 1e-10

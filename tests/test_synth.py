"""Seeded input generators: determinism and the structural properties the method assumes."""

import numpy as np

from synth import crystal_for, frequencies, gset_sorted, fcc_lattice
from synth.configs import closed_shell_counts


def test_deterministic():
    a = crystal_for("c1_small")
    b = crystal_for("c1_small")
    for x, y in zip(a.coef, b.coef):
        assert np.array_equal(x, y)
    for x, y in zip(a.eps, b.eps):
        assert np.array_equal(x, y)


def test_orbitals_orthonormal_and_sorted():
    cr = crystal_for("c1_small")
    for c, e in zip(cr.coef, cr.eps):
        assert np.abs(c @ c.conj().T - np.eye(c.shape[0])).max() < 1e-12
        assert np.all(np.diff(e[:cr.nocc]) >= 0) and np.all(np.diff(e[cr.nocc:]) >= 0)
    # gap after the scissor
    assert min(e[cr.nocc] for e in cr.eps) - max(e[cr.nocc - 1] for e in cr.eps) >= 0.05 - 1e-12


def test_gset_shells_and_frequencies():
    lat = fcc_lattice(10.26)
    g = gset_sorted(lat, 59)
    assert np.all(g[0] == 0)
    g2 = np.einsum("ij,ij->i", g @ lat.bvec, g @ lat.bvec) / lat.unit ** 2
    assert np.allclose(sorted(set(np.round(g2, 6))), [0, 3, 4, 8, 11, 12])
    assert closed_shell_counts(150, 900)[0] == 169
    w = frequencies(2)
    assert np.allclose(w, [0.0, 1.0])


def test_pairs_umklapp_consistent():
    cr = crystal_for("c1_small")
    for ik, ikp, g0 in cr.pairs:
        assert np.allclose(cr.kf[ik] - cr.qf, cr.kf[ikp] + g0)


def test_oracle_matches_stored_c1_record():
    import os
    from oracle.pipeline import epsinv_crystal
    rec = np.load(os.path.join(os.path.dirname(__file__), "golden", "c1_oracle.npz"))
    E, chi = epsinv_crystal(crystal_for("c1"))
    assert np.abs(E - rec["epsinv"]).max() < 1e-12
    assert np.abs(chi - rec["chi0"]).max() < 1e-12 * np.abs(rec["chi0"]).max()

"""Workload specifications for the five benchmark crystals and reduced test cases.

c1  plain FP64: fcc, 4 k-points {Gamma, X_x, X_y, X_z}, q = X_z, 8 occ + 24 empty,
    16^3 grid, NG = 59 (six closed shells), 2 imaginary frequencies.
c2  plain vs split precision: 4x4x4 k, q = b1/4, 16 occ + 200 empty, 36^3, NG = 400, 8 freqs.
c3  batched: 3x3x3 k, all 27 q, 32 occ + 400 empty, 48^3, NG per q from the closed-shell
    counts in [150, 900], 16 freqs.
c4  learned tail: c1 family on a 20^3 grid (N_pw ~ 1100), 8 occ + 1000 empty (full) / 100 (truncated),
    NG = 59, 8 freqs; train seeds 1000..1063, held-out 2000..2015.
c5  large cell: 32-site simple-cubic supercell, 2x2x2 k, q = b1/2, 128 occ + 2000 empty
    (200 explicit for the learned tail), 72^3, NG = 3000, 16 freqs (c5_small: the same cell, G-set and grid with k = {Gamma, b1/2},
    N_pw ~ 1500, 200 empty bands, 4 freqs).
"""

from __future__ import annotations

import numpy as np

from .crystal import (fcc_lattice, shell_potential, supercell_potential, ecut_for_npw,
                      kgrid_gamma, make_crystal, gset_sorted)

A_FCC = 10.26

FCC4 = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], float)

CONFIGS = {
    "c1": dict(lattice="fcc", kset="fcc4", q=(.5, .5, 0.), nocc=8, nempty=24, grid=16,
               npw=400, ng=59, nw=2, seed=1),
    "c2": dict(lattice="fcc", kset=4, q=(.25, 0., 0.), nocc=16, nempty=200, grid=36,
               npw=540, ng=400, nw=8, seed=2),
    "c3": dict(lattice="fcc", kset=3, q="all", nocc=32, nempty=400, grid=48,
               npw=900, ng=(150, 900), nw=16, seed=3),
    "c4": dict(lattice="fcc", kset="fcc4", q=(.5, .5, 0.), nocc=8, nempty=1000, ntrunc=100,
               grid=20, npw=1100, ng=59, nw=8, seed=1000),
    "c5": dict(lattice="sc32", kset=2, q=(.5, 0., 0.), nocc=128, nempty=2000, ntrunc=200, grid=72,
               npw=4000, ng=3000, nw=16, seed=5),
}

# Reduced variants used by tests: same families, sizes the oracle finishes in seconds.
CONFIGS["c1_small"] = dict(CONFIGS["c1"], npw=200, nempty=12)
CONFIGS["c2_small"] = dict(CONFIGS["c2"], kset=2, q=(.5, 0., 0.), nocc=4, nempty=28,
                           grid=20, npw=180, ng=89, nw=3)
CONFIGS["c4_small"] = dict(CONFIGS["c4"], grid=16, npw=300, nempty=120, ntrunc=20, nw=4)
# large cell at its real G-set (NG = 3000) and grid, one k-pair and its partner
# (Gamma and b1/2), a smaller plane-wave sphere and 200 empty bands
CONFIGS["c5_small"] = dict(CONFIGS["c5"], kset=((0., 0., 0.), (.5, 0., 0.)), npw=1500, nempty=200, nw=4)


def closed_shell_counts(lo: int, hi: int):
    """fcc Gamma-centred closed-shell G-set sizes in [lo, hi]."""
    lat = fcc_lattice(A_FCC)
    m = gset_sorted(lat, 4 * hi)
    g = m @ lat.bvec
    g2 = np.round(np.einsum("ij,ij->i", g, g) / lat.unit ** 2, 6)
    counts = [int(np.sum(g2 <= s)) for s in np.unique(g2)]
    return [c for c in counts if lo <= c <= hi]


def _kset(spec):
    ks = spec["kset"]
    if isinstance(ks, str) and ks == "fcc4":
        return FCC4.copy()
    if isinstance(ks, (list, tuple)):
        return np.array(ks, float).reshape(-1, 3)
    return kgrid_gamma(int(ks))


def crystal_for(name: str, seed: int = None, q=None, potential_zero: bool = False,
                nb_all: bool = False, progress=None, **over):
    """Build the crystal for a named workload (deterministic in the seed)."""
    spec = dict(CONFIGS[name], **over)
    seed = spec["seed"] if seed is None else seed
    kf = _kset(spec)
    qf = np.array(spec["q"] if q is None else q, float)
    grid = spec["grid"]
    grid = (grid,) * 3 if np.isscalar(grid) else tuple(grid)
    if spec["lattice"] == "fcc":
        lat = fcc_lattice(A_FCC)
        pot = shell_potential(lat, seed, zero=potential_zero)
    else:
        lat, pot = supercell_potential(A_FCC, seed)
    ecut = spec.get("ecut") or ecut_for_npw(lat, spec["npw"])
    ng = spec["ng"]
    if not np.isscalar(ng):
        choices = closed_shell_counts(*ng)
        ng = int(choices[np.random.default_rng(seed).integers(len(choices))])
    nb = None if nb_all else spec["nocc"] + spec["nempty"]
    cr = make_crystal(lat, pot, kf, qf, grid, ecut, spec["nocc"], nb, ng, spec["nw"], seed,
                      scissor_min=None if nb_all else 0.05, progress=progress)
    cr.meta = dict(name=name, spec=spec)
    return cr


def crystal_q_set(name: str = "c3", seed: int = None, nq: int = None, **over):
    """One crystal per q of the k-grid (all q = k-differences), sharing the orbitals.

    The G-set size of each q is a closed-shell count drawn with seed + iq from the
    configured range, so the set has uneven G-set sizes.
    """
    from dataclasses import replace
    from .crystal import find_pairs
    spec = dict(CONFIGS[name], **over)
    seed = spec["seed"] if seed is None else seed
    kf = _kset(spec)
    qs = kf.copy() if spec["q"] == "all" else np.array([spec["q"]], float)
    if nq is not None:
        qs = qs[:nq]
    base = crystal_for(name, seed=seed, q=qs[0], **over)
    lo, hi = spec["ng"] if not np.isscalar(spec["ng"]) else (spec["ng"], spec["ng"])
    choices = closed_shell_counts(lo, hi) if lo != hi else [lo]
    from .crystal import alias_extents
    out = []
    for iq, q in enumerate(qs):
        ng = int(choices[np.random.default_rng(seed + iq).integers(len(choices))])
        cr = replace(base, qf=np.asarray(q, float), pairs=find_pairs(base.kf, np.asarray(q, float)),
                     gmill=gset_sorted(base.lat, ng), meta=dict(base.meta, iq=iq))
        for ik, ikp, g0 in cr.pairs:
            ext = alias_extents(cr.grid, cr.mill[ik], cr.mill[ikp], cr.gmill, g0)
            if np.any(ext >= np.array(cr.grid)):
                raise ValueError(f"q #{iq}: grid {cr.grid} aliases (reach {ext})")
        out.append(cr)
    return out

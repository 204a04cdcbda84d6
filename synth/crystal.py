"""Seeded model crystals: geometry, plane-wave spheres, Hamiltonian eigenpairs.

The method consumes Kohn-Sham energies and plane-wave wavefunctions from a DFT
code (the interfaces section of the paper). No DFT data exists here, so a model
Hamiltonian stands in:

    H_k(G, G') = 1/2 |k+G|^2 delta_GG' + V(G - G'),

diagonalised on the sphere 1/2|k+G|^2 <= E_cut. Orbitals are the eigenvectors,
normalised to sum_G |c(G)|^2 = 1, multiplied by a seeded random phase per
(k, band) so that the coefficients are genuinely complex and the band gauge is
arbitrary, as it is for independently diagonalised k-points.

Conventions
-----------
* A reciprocal vector is a Miller triple m with G = m @ bvec (rows of bvec are
  the primitive reciprocal vectors b_i). Its index on an N1 x N2 x N3 FFT grid
  is m mod N; the real-space grid point j sits at r = sum_i (j_i/N_i) a_i, so
  G.r = 2 pi sum_i m_i j_i / N_i.
* k-points and q are given in fractional coordinates of the b_i.
* For a transition pair, k - q = k' + G0 with k' a stored k-point and G0 an
  integer Miller triple (umklapp).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg

from .rand import rng

TWO_PI = 2.0 * np.pi


@dataclass
class Lattice:
    avec: np.ndarray  # (3,3) rows are real-space primitive vectors, bohr
    bvec: np.ndarray  # (3,3) rows are reciprocal primitive vectors, 1/bohr
    omega: float      # primitive-cell volume, bohr^3
    unit: float       # natural reciprocal length unit (2 pi / a), 1/bohr


def fcc_lattice(a: float) -> Lattice:
    avec = 0.5 * a * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=np.float64)
    t = TWO_PI / a
    bvec = t * np.array([[-1, 1, 1], [1, -1, 1], [1, 1, -1]], dtype=np.float64)
    return Lattice(avec, bvec, abs(np.linalg.det(avec)), t)


def sc_lattice(L: float) -> Lattice:
    avec = L * np.eye(3)
    t = TWO_PI / L
    return Lattice(avec, t * np.eye(3), L ** 3, t)


def _miller_box(lat: Lattice, radius: float) -> np.ndarray:
    """All Miller triples whose |G| could be <= radius (a superset)."""
    # |m_i| = |G . a_i| / 2pi <= radius |a_i| / 2pi
    lim = [int(np.floor(radius * np.linalg.norm(lat.avec[i]) / TWO_PI)) + 1 for i in range(3)]
    ax = [np.arange(-l, l + 1) for l in lim]
    m = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1).reshape(-1, 3)
    return m.astype(np.int64)


def _sort_key(m: np.ndarray, g2: np.ndarray) -> np.ndarray:
    """Order by |G|^2 (rounded to remove float noise), then Miller lexicographic."""
    g2r = np.round(g2, 9)
    return np.lexsort((m[:, 2], m[:, 1], m[:, 0], g2r))


def miller_sphere(lat: Lattice, kf: np.ndarray, ecut: float) -> np.ndarray:
    """Miller triples with 1/2 |k+G|^2 <= ecut, sorted by (|k+G|^2, m)."""
    kc = np.asarray(kf, float) @ lat.bvec
    radius = np.sqrt(2.0 * ecut) + np.linalg.norm(kc)
    m = _miller_box(lat, radius)
    kg = kc[None, :] + m @ lat.bvec
    g2 = np.einsum("ij,ij->i", kg, kg)
    sel = 0.5 * g2 <= ecut * (1.0 + 1e-12)
    m, g2 = m[sel], g2[sel]
    return m[_sort_key(m, g2)].astype(np.int32)


def gset_sorted(lat: Lattice, ng: int) -> np.ndarray:
    """First ng Gamma-centred reciprocal vectors sorted by (|G|^2, Miller triple)."""
    radius = lat.unit
    while True:
        m = _miller_box(lat, radius)
        g = m @ lat.bvec
        g2 = np.einsum("ij,ij->i", g, g)
        inside = g2 <= radius ** 2
        if inside.sum() > ng:
            break
        radius *= 1.5
    m, g2 = m[inside], g2[inside]
    return m[_sort_key(m, g2)][:ng].astype(np.int32)


def ecut_for_npw(lat: Lattice, npw: int) -> float:
    """Smallest cutoff whose Gamma sphere holds at least npw vectors (whole shells)."""
    radius = lat.unit
    while True:
        m = _miller_box(lat, radius)
        g = m @ lat.bvec
        g2 = np.sort(np.einsum("ij,ij->i", g, g))
        if np.sum(g2 <= radius ** 2) > npw:
            break
        radius *= 1.3
    return 0.5 * g2[npw - 1] * (1.0 + 1e-10)


def kgrid_gamma(n: int) -> np.ndarray:
    """Gamma-centred n x n x n grid, fractional coordinates folded into [-1/2, 1/2)."""
    i = (np.arange(n) + n // 2) % n - n // 2
    k = np.stack(np.meshgrid(i, i, i, indexing="ij"), axis=-1).reshape(-1, 3)
    return k.astype(np.float64) / n


def frequencies(nw: int) -> np.ndarray:
    """Imaginary frequencies omega_j = (1 Ha) tan(pi j / (2 nw)), j = 0..nw-1."""
    j = np.arange(nw, dtype=np.float64)
    return np.tan(np.pi * j / (2.0 * nw))


# ----------------------------------------------------------------------------
# Model potentials
# ----------------------------------------------------------------------------

FCC_SHELLS = (3.0, 4.0, 8.0, 11.0, 12.0, 16.0)  # |G|^2 in units of (2pi/a)^2


@dataclass
class ShellPotential:
    """Real, inversion-symmetric V(G) = V_s on the s-th Gamma-centred shell."""
    lat: Lattice
    shells: Tuple[float, ...]
    values: np.ndarray

    def __call__(self, dm: np.ndarray) -> np.ndarray:
        g = dm.astype(np.float64) @ self.lat.bvec
        g2 = np.einsum("...i,...i->...", g, g) / self.lat.unit ** 2
        v = np.zeros(g2.shape, dtype=np.complex128)
        for s, val in zip(self.shells, self.values):
            v[np.abs(g2 - s) < 1e-6] = val
        return v


def shell_potential(lat: Lattice, seed: int, amp: float = 0.3,
                    zero: bool = False) -> ShellPotential:
    vals = np.zeros(len(FCC_SHELLS)) if zero else amp * rng(seed).uniform(-1.0, 1.0, len(FCC_SHELLS))
    return ShellPotential(lat, FCC_SHELLS, vals)


@dataclass
class SupercellPotential:
    """V(G) = (1/N_at) sum_a exp(-i G.tau_a) v(|G|) for a displaced-site supercell."""
    lat: Lattice
    tau: np.ndarray        # (N_at, 3) Cartesian positions, bohr
    knots_g: np.ndarray    # |G| knots (1/bohr)
    knots_v: np.ndarray    # v at the knots (Ha)
    gmax: float

    def __call__(self, dm: np.ndarray) -> np.ndarray:
        from scipy.interpolate import CubicSpline
        g = dm.astype(np.float64) @ self.lat.bvec
        gn = np.sqrt(np.einsum("...i,...i->...", g, g))
        spl = CubicSpline(self.knots_g, self.knots_v, bc_type="clamped")
        v = np.where((gn > 1e-12) & (gn <= self.gmax), spl(np.minimum(gn, self.gmax)), 0.0)
        phase = np.exp(-1j * np.einsum("...i,ai->...a", g, self.tau)).mean(axis=-1)
        return v * phase


def supercell_potential(a_fcc: float, seed: int, sigma: float = 0.1) -> Tuple[Lattice, SupercellPotential]:
    """Simple-cubic 2a supercell holding 32 fcc sites with seeded displacements."""
    L = 2.0 * a_fcc
    lat = sc_lattice(L)
    base = 0.5 * a_fcc * np.array([[0, 0, 0], [0, 1, 1], [1, 0, 1], [1, 1, 0]], float)
    cells = np.array([[i, j, k] for i in range(2) for j in range(2) for k in range(2)], float) * a_fcc
    tau = (cells[:, None, :] + base[None, :, :]).reshape(-1, 3)
    tau = tau + rng(seed).normal(0.0, sigma, tau.shape)
    fcc = fcc_lattice(a_fcc)
    shell_v = shell_potential(fcc, seed).values
    gk = np.sqrt(np.array((0.0,) + FCC_SHELLS)) * fcc.unit
    vk = np.concatenate([[shell_v[0]], shell_v])
    gmax = np.sqrt(FCC_SHELLS[-1]) * fcc.unit
    return lat, SupercellPotential(lat, tau, gk, vk, gmax)


# ----------------------------------------------------------------------------
# Crystal
# ----------------------------------------------------------------------------

@dataclass
class Crystal:
    lat: Lattice
    kf: np.ndarray                 # (nk, 3) fractional k-points
    qf: np.ndarray                 # (3,) fractional q
    grid: Tuple[int, int, int]
    ecut: float
    nocc: int
    mill: List[np.ndarray]         # per k: (npw_k, 3) int32
    coef: List[np.ndarray]         # per k: (nb_k, npw_k) complex128, unit-norm rows
    eps: List[np.ndarray]          # per k: (nb_k,) float64 (scissor applied to empty bands)
    gmill: np.ndarray              # (ng, 3) int32 chi0 G-set
    omegas: np.ndarray             # (nw,) imaginary frequencies in Ha
    pairs: List[Tuple[int, int, np.ndarray]]  # (ik, ik', G0) with k_ik - q = k_ik' + G0
    scissor: float = 0.0
    seed: int = 0
    meta: dict = field(default_factory=dict)
    nocc_k: Optional[List[int]] = None   # per-k occupied count (defaults to nocc everywhere)

    def nocc_at(self, ik: int) -> int:
        return self.nocc if self.nocc_k is None else int(self.nocc_k[ik])

    @property
    def nk(self) -> int:
        return len(self.kf)

    @property
    def q0(self) -> bool:
        return bool(np.all(np.abs(self.qf) < 1e-12))

    def kcart(self, ik: int) -> np.ndarray:
        return self.kf[ik] @ self.lat.bvec

    def qcart(self) -> np.ndarray:
        return self.qf @ self.lat.bvec

    def ntrans(self, nempty: Optional[int] = None) -> int:
        tot = 0
        for ik, ikp, _ in self.pairs:
            nc = self.coef[ik].shape[0] - self.nocc_at(ik)
            if nempty is not None:
                nc = min(nc, nempty)
            tot += self.nocc_at(ikp) * nc
        return tot


def find_pairs(kf: np.ndarray, qf: np.ndarray) -> List[Tuple[int, int, np.ndarray]]:
    """For each k, the stored k' and integer G0 with k - q = k' + G0."""
    out = []
    for ik in range(len(kf)):
        kmq = kf[ik] - qf
        found = None
        for ikp in range(len(kf)):
            d = kmq - kf[ikp]
            if np.all(np.abs(d - np.round(d)) < 1e-9):
                found = (ik, ikp, np.round(d).astype(np.int32))
                break
        if found is None:
            raise ValueError(f"k - q for k #{ik} is not in the k-set (set not closed)")
        out.append(found)
    return out


def hamiltonian(lat: Lattice, kf: np.ndarray, mill: np.ndarray, pot) -> np.ndarray:
    kg = (np.asarray(kf, float)[None, :] + mill) @ lat.bvec
    # V(G - G') depends only on the Miller difference: evaluate it once per distinct
    # difference (a dense box of them) and gather
    lo = mill.min(0).astype(np.int64)
    span = mill.max(0).astype(np.int64) - lo
    size = 2 * span + 1
    box = np.stack(np.meshgrid(*[np.arange(-s, s + 1) for s in span], indexing="ij"), axis=-1).reshape(-1, 3)
    vbox = pot(box)
    m = mill.astype(np.int64)
    flat = ((m[:, 0] * size[1] + m[:, 1]) * size[2] + m[:, 2])
    base = (span[0] * size[1] + span[1]) * size[2] + span[2]
    H = vbox[flat[:, None] - flat[None, :] + base]
    H[np.diag_indices_from(H)] += 0.5 * np.einsum("ij,ij->i", kg, kg)
    return H


def _solve(H: np.ndarray, nb: int) -> Tuple[np.ndarray, np.ndarray]:
    n = H.shape[0]
    if nb >= n:
        w, v = scipy.linalg.eigh(H)
    else:
        w, v = scipy.linalg.eigh(H, subset_by_index=[0, nb - 1], driver="evr")
    return w, v


def alias_extents(grid, mill_c: np.ndarray, mill_v: np.ndarray, gmill: np.ndarray,
                  g0: np.ndarray) -> np.ndarray:
    """Per-axis worst-case reach of the wrap-around correlation; must be < N."""
    dhi = mill_c.max(0).astype(np.int64) - mill_v.min(0)
    dlo = mill_c.min(0).astype(np.int64) - mill_v.max(0)
    e = gmill.astype(np.int64) - g0[None, :]
    reach = np.maximum(dhi - e.min(0), e.max(0) - dlo)
    span = np.maximum(mill_c.max(0) - mill_c.min(0), mill_v.max(0) - mill_v.min(0))
    return np.maximum(reach, span)


def make_crystal(lat: Lattice, pot, kf: np.ndarray, qf: np.ndarray, grid, ecut: float,
                 nocc: int, nb: Optional[int], ng: int, nw: int, seed: int,
                 scissor_min: Optional[float] = 0.05, phases: bool = True,
                 check_alias: bool = True, nocc_k: Optional[Sequence[int]] = None, progress=None) -> Crystal:
    kf = np.asarray(kf, float).reshape(-1, 3)
    qf = np.asarray(qf, float).reshape(3)
    pairs = find_pairs(kf, qf)
    g = rng(seed + 7919)
    mills, coefs, epss = [], [], []
    for ik in range(len(kf)):
        m = miller_sphere(lat, kf[ik], ecut)
        H = hamiltonian(lat, kf[ik], m, pot)
        nbk = m.shape[0] if nb is None else nb
        if nbk > m.shape[0]:
            raise ValueError(f"{nbk} bands requested but the sphere holds {m.shape[0]} plane waves")
        w, v = _solve(H, nbk)
        c = np.ascontiguousarray(v.T).astype(np.complex128)
        if phases:
            c *= np.exp(1j * g.uniform(0.0, TWO_PI, nbk))[:, None]
        mills.append(m)
        coefs.append(c)
        epss.append(w.astype(np.float64))
        if progress:
            progress(f"k-point {ik + 1}/{len(kf)}: {m.shape[0]} plane waves, {nbk} bands")
    shift = 0.0
    occ = [nocc] * len(kf) if nocc_k is None else list(nocc_k)
    if scissor_min is not None:
        vbm = max(e[o - 1] for e, o in zip(epss, occ))
        cbm = min(e[o] for e, o in zip(epss, occ) if e.shape[0] > o)
        gap = cbm - vbm
        if gap < scissor_min:
            shift = scissor_min - gap
            for e, o in zip(epss, occ):
                e[o:] += shift
    gm = gset_sorted(lat, ng)
    cr = Crystal(lat=lat, kf=kf, qf=qf, grid=tuple(int(x) for x in grid), ecut=ecut, nocc=nocc,
                 mill=mills, coef=coefs, eps=epss, gmill=gm, omegas=frequencies(nw),
                 pairs=pairs, scissor=shift, seed=seed,
                 nocc_k=None if nocc_k is None else [int(x) for x in nocc_k])
    if check_alias:
        for ik, ikp, g0 in pairs:
            ext = alias_extents(cr.grid, mills[ik], mills[ikp], gm, g0)
            if np.any(ext >= np.array(cr.grid)):
                raise ValueError(f"FFT grid {cr.grid} aliases for pair {ik},{ikp}: reach {ext}")
    return cr

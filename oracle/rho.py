"""Oscillator strengths rho_{cv k}(q, G) in FP64. TEST INFRASTRUCTURE (oracle).

Definition (Linear Response section, Eq. rhotw):

    rho_{nm k}(q, G) = < n k | exp(i (q+G).r) | m k-q >,

with the conduction (empty) state n = c at k, the valence (occupied) state
m = v at k - q, and the bracket the cell-averaged integral (1/Omega) int_Omega.
With psi_{nk}(r) = exp(ik.r) sum_G c_nk(G) exp(iG.r) and k - q = k' + G0 the
phase factors cancel and

    rho(G) = (1/N_r) sum_r conj(u_c(r)) u_{v,k'}(r) exp(i (G - G0).r)       (FFT route)
           = sum_{G2} conj(c_c(G + G2 - G0)) c_{v,k'}(G2)                      (direct route)

The paper evaluates the first form: the Fourier transform of the real-space
product of the two wavefunctions. The second is the definition written out
and serves to pin the first.
"""

from __future__ import annotations

import numpy as np
import scipy.fft

# FFTs on every host core (the same transform as numpy's; threads only split the batch)
FFT_WORKERS = -1


def _lookup(mill: np.ndarray):
    """Hash of Miller triples -> row index (dict; plain and obviously correct)."""
    return {tuple(int(x) for x in m): i for i, m in enumerate(mill)}


def rho_direct(coef_c, mill_c, coef_v, mill_v, gmill, g0):
    """Direct plane-wave convolution; returns rho[v, c, G] (complex128).

    coef_c: (nc, npw_c) conduction coefficients at k on sphere mill_c
    coef_v: (nv, npw_v) valence coefficients at k' on sphere mill_v
    Terms whose G + G2 - G0 falls outside the k sphere are zero (the orbital
    has no such component).
    """
    look = _lookup(mill_c)
    ng = gmill.shape[0]
    nc, nv = coef_c.shape[0], coef_v.shape[0]
    out = np.zeros((nv, nc, ng), dtype=np.complex128)
    for ig in range(ng):
        target = mill_v.astype(np.int64) + (gmill[ig].astype(np.int64) - g0)[None, :]
        idx = np.array([look.get(tuple(int(x) for x in t), -1) for t in target])
        ok = idx >= 0
        # sum over G2 of conj(c_c(G+G2-G0)) c_v(G2)
        out[:, :, ig] = coef_v[:, ok] @ np.conj(coef_c[:, idx[ok]]).T
    return out


def orbitals_real_space(coef, mill, grid):
    """u(r) = sum_G c(G) exp(iG.r) on the grid, for each band: (nb, N1, N2, N3)."""
    grid = tuple(int(x) for x in grid)
    nr = grid[0] * grid[1] * grid[2]
    box = np.zeros((coef.shape[0],) + grid, dtype=np.complex128)
    ix = tuple(np.mod(mill[:, a], grid[a]) for a in range(3))
    box[:, ix[0], ix[1], ix[2]] = coef
    # numpy ifftn carries exp(+i) and 1/N_r; multiply back by N_r
    return scipy.fft.ifftn(box, axes=(1, 2, 3), workers=FFT_WORKERS) * nr


def rho_fft(coef_c, mill_c, coef_v, mill_v, gmill, g0, grid):
    """FFT route of Eq. (rhotw): transform of the real-space product; rho[v, c, G]."""
    grid = tuple(int(x) for x in grid)
    uc = orbitals_real_space(coef_c, mill_c, grid)
    uv = orbitals_real_space(coef_v, mill_v, grid)
    sel = tuple(np.mod(gmill[:, a].astype(np.int64) - g0[a], grid[a]) for a in range(3))
    nc, nv, ng = coef_c.shape[0], coef_v.shape[0], gmill.shape[0]
    out = np.zeros((nv, nc, ng), dtype=np.complex128)
    for v in range(nv):
        prod = np.conj(uc) * uv[v][None]
        # (1/N_r) sum_r p(r) exp(+i(G-G0).r)
        f = scipy.fft.ifftn(prod, axes=(1, 2, 3), workers=FFT_WORKERS)
        out[v] = f[:, sel[0], sel[1], sel[2]]
    return out


def rho_head_q0(coef_c, e_c, coef_v, e_v, mill, kcart, bvec, qhat):
    """q -> 0 limit of the G = 0 column, divided by |q| (Eq. dip, G-space v approach).

    For a local Hamiltonian [r, V] = 0, so dH/dk = k + G in the plane-wave basis and
    k.p perturbation theory gives, for c != v,

        rho_cv(q -> 0, 0) / |q| = qhat . sum_G conj(c_c(G)) (k+G) c_v(G) / (e_c - e_v).

    Returns rhohat[v, c]. Requires e_c != e_v for every pair.
    """
    kg = kcart[None, :] + mill.astype(np.float64) @ bvec
    proj = kg @ np.asarray(qhat, float)                    # qhat . (k+G)
    num = (coef_v * proj[None, :]) @ np.conj(coef_c).T     # [v, c] = sum_G c_v (q.(k+G)) c_c*
    den = e_c[None, :] - e_v[:, None]
    return num / den

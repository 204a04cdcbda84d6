"""Independent-particle response chi0 at imaginary frequencies. TEST INFRASTRUCTURE (oracle).

Eq. (X_IP) with the split of Appendix A (Eq. X_IP_split): a frequency-independent
outer product R_t(G, G') = pref rho_t(G) conj(rho_t(G')) per transition t, times a
frequency factor F_t(omega). For an occupied state v (f = 1) at k - q and an empty
state c (f = 0) at k with Delta_t = e_{c,k} - e_{v,k-q} > 0, the pole pair of a
density response is

    F_t(omega) = 1/(omega - Delta_t + i eta) - 1/(omega + Delta_t - i eta),

which at omega = i w, eta = 0 is  -2 Delta_t / (w^2 + Delta_t^2)  (real, negative), so

    chi0_GG'(q, i w) = -pref sum_t [2 Delta_t / (w^2 + Delta_t^2)] rho_t(G) conj(rho_t(G')),

pref = f_s / (N_k Omega), f_s = 2. Reading of the printed bracket: as typeset its
sign gives a positive static response, which a density response cannot be; the
form above is negative semidefinite. The index order rho(G) rho*(G') follows
Eq. (X_IP) (the swapped indices in Eq. X_IP_split2 are taken as a typo).
"""

from __future__ import annotations

import numpy as np


SPIN_FACTOR = 2.0   # f_s: spin-unpolarised, two electrons per occupied band


def cell_volume(avec) -> float:
    """Omega = |det(a1, a2, a3)|, the volume of the primitive cell (rows of avec, bohr)."""
    return float(abs(np.linalg.det(np.asarray(avec, dtype=np.float64))))


def chi0_prefactor(nk: int, avec) -> float:
    """pref = f_s / (N_k Omega) of Eq. (X_IP): the spin factor over the number of
    k-points times the cell volume (the Brillouin-zone sum as an average)."""
    return SPIN_FACTOR / (int(nk) * cell_volume(avec))


def crystal_prefactor(cr) -> float:
    """pref of a crystal: its k-point count and its lattice vectors."""
    return chi0_prefactor(len(cr.kf), cr.lat.avec)


def pole_weights(dE: np.ndarray, w: float) -> np.ndarray:
    """2 Delta / (w^2 + Delta^2) for each transition (the magnitude of -F_t(i w))."""
    dE = np.asarray(dE, dtype=np.float64)
    return 2.0 * dE / (w * w + dE * dE)


def chi0_from_rho(M: np.ndarray, dE: np.ndarray, omegas, pref: float) -> np.ndarray:
    """chi0[w, G, G'] from the transition matrix M[t, G] (complex128, full matrix zgemm)."""
    M = np.asarray(M, dtype=np.complex128)
    out = np.empty((len(omegas), M.shape[1], M.shape[1]), dtype=np.complex128)
    for j, w in enumerate(omegas):
        wt = pole_weights(dE, w)
        # sum_t wt_t M[t, G] conj(M[t, G'])
        out[j] = -pref * (M.T * wt[None, :]) @ np.conj(M)
    return out


def pole_factor_real_axis(dE, omega, eta: float):
    """F_t(omega) = 1/(omega - Delta_t + i eta) - 1/(omega + Delta_t - i eta) (complex).

    The time-ordered form of the bracket of Eq. (X_IP) with the sign reading above
    (poles at Delta - i eta and -Delta + i eta). omega may be complex: omega = i w with
    eta = 0 gives the imaginary-axis factor -2 Delta / (w^2 + Delta^2)."""
    dE = np.asarray(dE, dtype=np.float64)
    return 1.0 / (omega - dE + 1j * eta) - 1.0 / (omega + dE - 1j * eta)


def chi0_real_axis(M: np.ndarray, dE: np.ndarray, omegas, eta: float, pref: float) -> np.ndarray:
    """chi0[w, G, G'] = pref sum_t F_t(omega_w) M[t, G] conj(M[t, G']) at real (or complex)
    frequencies: Eq. (X_IP) with every transition its own pole group (Appendix A with
    the degeneracy threshold at zero). Not Hermitian: chi0 = A + i B with A and B the
    Hermitian sums weighted by Re F and Im F."""
    M = np.asarray(M, dtype=np.complex128)
    out = np.empty((len(omegas), M.shape[1], M.shape[1]), dtype=np.complex128)
    for j, w in enumerate(omegas):
        F = pole_factor_real_axis(dE, w, eta)
        out[j] = pref * (M.T * F[None, :]) @ np.conj(M)
    return out

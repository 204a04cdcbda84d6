"""Plasmon-pole screening and GW self-energy matrix elements. TEST INFRASTRUCTURE (oracle).

Quasi-particle corrections section: the split of Sigma into a bare exchange and a
screened correlation part, Eq. (sigma_c), Eq. (I_c) and the screened interaction of
Eq. (W_def), and the plasmon-pole paragraph of the Full frequency GW subsection
(Godby-Needs: the model is fixed by the inverse dielectric matrix at omega = 0 and at
one imaginary frequency i omega_p, 1 Ha by default; the frequency integral of
Eq. (sigma_c) then has a closed form). The paper prints neither the model nor the
closed form; the readings taken here:

* Model. Every element of X = eps~^-1 - 1 (the symmetrised inverse of the
  Linear Algebra subsection) carries one pole pair,
      X_GG'(omega) = R_GG' [1/(omega - Om_GG' + i0) - 1/(omega + Om_GG' - i0)],
  so X(i nu) = -2 R Om / (nu^2 + Om^2). The two samples fix it:
      Om^2 = omega_p^2 Xp / (X0 - Xp),   R = -X0 Om / 2,
  with X0 = X(0), Xp = X(i omega_p) and the principal square root. An element is
  fitted when Re(Xp conj(X0 - Xp)) > 0 (that is Re Om^2 > 0, so the pole lies off
  the imaginary axis on the right side); any other element keeps its static value
  with Om = omega_p, R = -X0 omega_p / 2.
* Coulomb factor. W_c = v^1/2 X v^1/2 (Eq. W_def with the symmetrised inverse), with
  v^1/2_G = sqrt(4 pi) / |q + G| given per G. At q = 0 the caller passes 0 for the
  G = 0 entry (the wings, odd in q, average to zero over the small cell around
  q = 0) and the cell average of 4 pi / q^2 as `head`, which then multiplies the
  (0, 0) element.
* Correlation (diagonal elements only). With the pole form the integral of
  Eq. (sigma_c) over the screened part gives, for a state n at k,
      Sigma_c,nn(z) = pref sum_{q,m} sum_{G,G'} rho_nm(q,G) conj(rho_nm(q,G')) Wr_GG'
                      [ f_m / (z - e_m + Om_GG' - i eta) + (1 - f_m) / (z - e_m - Om_GG' + i eta) ],
  Wr = residue of W_c (R times the Coulomb factor), e_m and f_m (in [0, 1], per spin)
  the energy and occupation of band m at k - q, pref = 1 / (N_k Omega). The index
  order rho_nm(G) conj(rho_n'm(G')) follows Eq. (I_c). z may be complex: with
  eta = 0 and z = i nu this is the imaginary-axis self-energy.
* Exchange. Sigma_x,nn = -pref sum_{q,m} f_m sum_G |rho_nm(q,G)|^2 v_G.

Pins (tests/test_oracle_sigma.py): the fit reproduces X at both samples and recovers
the parameters of an exact one-pole input; Sigma_c at z = i nu equals the frequency
integral -(1/2 pi) int G(i nu + i w) W_c(i w) dw done by quadrature (the GW product
on the imaginary axis); Sigma_x of plane-wave orbitals equals the Fock exchange
-pref sum 4 pi / |p_n - p_m|^2 over the occupied plane waves, summed directly.
"""

from __future__ import annotations

import numpy as np

from .chi0 import cell_volume


def ppa_fit(einv0, einvp, omega_p: float):
    """Plasmon-pole parameters (R, Om) of every element from eps~^-1 at 0 and i omega_p."""
    einv0 = np.asarray(einv0, np.complex128)
    einvp = np.asarray(einvp, np.complex128)
    n = einv0.shape[0]
    eye = np.eye(n)
    X0 = einv0 - eye
    Xp = einvp - eye
    R = np.empty_like(X0)
    Om = np.empty_like(X0)
    for a in range(n):
        for b in range(n):
            x0, xp = X0[a, b], Xp[a, b]
            d = x0 - xp
            if xp.real * d.real + xp.imag * d.imag > 0.0:
                om = omega_p * np.sqrt(xp / d)
            else:
                om = complex(omega_p, 0.0)
            Om[a, b] = om
            R[a, b] = -x0 * om / 2.0
    return R, Om


def ppa_eval_imag(R, Om, nu: float):
    """X(i nu) of the pole model (used by the pins)."""
    return -2.0 * R * Om / (nu * nu + Om * Om)


def coulomb_factor(vsqrt, head=None):
    """v^1/2_G v^1/2_G', with the (0, 0) element replaced by `head` when given."""
    s = np.asarray(vsqrt, np.float64)
    c = np.outer(s, s)
    if head is not None:
        c[0, 0] = head
    return c


def sigma_c_ppa(rho, Wr, Om, e_m, f_m, z, eta: float, pref: float):
    """Sigma_c,nn(z_nj) for one q.

    rho[m, n, G] = rho_nm(q, G) (state n at k, band m at k - q); Wr, Om: [G, G'];
    e_m, f_m: [m]; z[n, j] complex. Returns [n, j] complex128.
    """
    rho = np.asarray(rho, np.complex128)
    nm, nn, ng = rho.shape
    z = np.asarray(z, np.complex128).reshape(nn, -1)
    out = np.zeros(z.shape, np.complex128)
    for n in range(nn):
        for m in range(nm):
            P = np.outer(rho[m, n], np.conj(rho[m, n])) * Wr   # rho(G) conj(rho(G')) Wr_GG'
            f = float(f_m[m])
            for j in range(z.shape[1]):
                D = f / (z[n, j] - e_m[m] + Om - 1j * eta) + (1.0 - f) / (z[n, j] - e_m[m] - Om + 1j * eta)
                out[n, j] += pref * np.sum(P * D)
    return out


def sigma_x(rho, f_m, vsqrt, head, pref: float):
    """Sigma_x,nn for one q: -pref sum_m f_m sum_G |rho_nm(G)|^2 v_G (real)."""
    rho = np.asarray(rho, np.complex128)
    v = np.asarray(vsqrt, np.float64) ** 2
    if head is not None:
        v = v.copy()
        v[0] = head
    nm, nn, _ = rho.shape
    out = np.zeros(nn)
    for n in range(nn):
        for m in range(nm):
            out[n] -= pref * float(f_m[m]) * np.sum(np.abs(rho[m, n]) ** 2 * v)
    return out


def sigma_prefactor(nk: int, avec) -> float:
    """pref = 1 / (N_k Omega): the q-sum of Eq. (sigma_c) as a Brillouin-zone average over
    the N_k points of the grid, with the cell volume from the lattice vectors. Sigma is per
    spin (f_m in [0, 1]), so there is no spin factor."""
    return 1.0 / (int(nk) * cell_volume(avec))


def coulomb_head_average(nk: int, omega: float) -> float:
    """Cell average of 4 pi / q^2 at q = 0, over the sphere whose volume is the
    Brillouin-zone share of one k-point, (2 pi)^3 / (N_k Omega) (a reading: the paper
    leaves the q = 0 treatment of Sigma to the Coulomb subsection's options)."""
    qc = (6.0 * np.pi ** 2 / (nk * omega)) ** (1.0 / 3.0)
    # int_0^qc 4 pi q^2 (4 pi / q^2) dq / (4/3 pi qc^3)
    return 16.0 * np.pi ** 2 * qc / (4.0 / 3.0 * np.pi * qc ** 3)


def sigma_kpoint(crs, einv_by_q, ik0: int, states, z, eta: float = 0.0, omega_p: float = 1.0):
    """Sigma_x and Sigma_c of the states n at k-point ik0, summed over the q of `crs`.

    crs: one crystal per q sharing the orbitals; einv_by_q[iq] = eps~^-1 at (0, i omega_p);
    the bands m at k - q are all the stored bands, occupied ones with f = 1.
    Returns (sigx [n], sigc [n, j])."""
    from .rho import rho_fft
    states = list(states)
    z = np.asarray(z, np.complex128).reshape(len(states), -1)
    sx = np.zeros(len(states))
    sc = np.zeros(z.shape, np.complex128)
    for cr, E in zip(crs, einv_by_q):
        ik, ikp, g0 = cr.pairs[ik0]
        assert ik == ik0
        nb = cr.coef[ikp].shape[0]
        rho = rho_fft(cr.coef[ik0][states], cr.mill[ik0], cr.coef[ikp], cr.mill[ikp], cr.gmill, g0, cr.grid)
        qg = (cr.qf @ cr.lat.bvec)[None, :] + cr.gmill.astype(np.float64) @ cr.lat.bvec
        nrm = np.sqrt(np.sum(qg * qg, axis=1))
        head = None
        assert np.all(cr.gmill[0] == 0)
        if cr.q0:
            s = np.zeros_like(nrm)
            s[1:] = np.sqrt(4.0 * np.pi) / nrm[1:]
            head = coulomb_head_average(cr.nk, cell_volume(cr.lat.avec))
        else:
            s = np.sqrt(4.0 * np.pi) / nrm
        R, Om = ppa_fit(E[0], E[1], omega_p)
        Wr = R * coulomb_factor(s, head)
        f = np.zeros(nb)
        f[:cr.nocc_at(ikp)] = 1.0
        pref = sigma_prefactor(cr.nk, cr.lat.avec)
        sx += sigma_x(rho, f, s, head, pref)
        sc += sigma_c_ppa(rho, Wr, Om, cr.eps[ikp], f, z, eta, pref)
    return sx, sc

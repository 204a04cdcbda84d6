"""Dyson inversion for the inverse dielectric matrix in FP64. TEST INFRASTRUCTURE (oracle).

Bare Coulomb potential v(q+G) = 4 pi / |q+G|^2 (Coulomb interaction subsection).
The RPA response solves Eq. (X_rpa) by a matrix inversion, Eq. (X_rpa_inv); the
dielectric matrix is eps = 1 - v chi0. With s_G = sqrt(4 pi) / |q+G| the
symmetrised matrix

    eps~ = I - diag(s) chi0 diag(s)

is Hermitian positive definite at imaginary frequencies (chi0 <= 0), and eps~^-1
is the matrix that Eq. (W_def) multiplies by 4 pi / (|q+G| |q+G'|) to give W.
The non-symmetric (I - v chi0)^-1 = diag(s) eps~^-1 diag(1/s) shares its diagonal.
At q = 0 the caller passes |q+G| = 1 for G = 0 and q-normalised head/wings, so
s_0 = sqrt(4 pi).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


def qpg_norms(bvec, qf, gmill) -> np.ndarray:
    """|q+G| in 1/bohr for the G-set (q and G in units of the reciprocal vectors, rows of
    bvec). At q = 0 the G = 0 entry is 1: the head and wings of chi0 there are the
    q-normalised limits (rho / |q|), so s_0 = sqrt(4 pi)."""
    qg = (np.asarray(qf, dtype=np.float64)[None, :] + np.asarray(gmill, dtype=np.float64)) @ np.asarray(bvec, float)
    n = np.sqrt(np.einsum("ij,ij->i", qg, qg))
    n[n < 1e-12] = 1.0
    return n


def crystal_qpg(cr) -> np.ndarray:
    return qpg_norms(cr.lat.bvec, cr.qf, cr.gmill)


def coulomb_sqrt(qpg: np.ndarray) -> np.ndarray:
    return np.sqrt(4.0 * np.pi) / np.asarray(qpg, dtype=np.float64)


def eps_tilde(chi0: np.ndarray, qpg: np.ndarray) -> np.ndarray:
    s = coulomb_sqrt(qpg)
    ng = chi0.shape[-1]
    return np.eye(ng)[None] - s[None, :, None] * chi0 * s[None, None, :]


def epsinv_sym(chi0: np.ndarray, qpg: np.ndarray, check: bool = True) -> np.ndarray:
    """eps~^-1 per frequency, by LU (numpy.linalg.inv) cross-checked with Cholesky."""
    et = eps_tilde(chi0, qpg)
    out = np.empty_like(et)
    for j in range(et.shape[0]):
        inv_lu = np.linalg.inv(et[j])
        if check:
            cf = scipy.linalg.cho_factor(et[j], lower=True)
            inv_ch = scipy.linalg.cho_solve(cf, np.eye(et.shape[-1]))
            err = np.linalg.norm(inv_lu - inv_ch) / np.linalg.norm(inv_lu)
            assert err < 1e-10, f"LU and Cholesky inverses disagree: {err}"
        out[j] = inv_lu
    return out


def epsinv_nonsym(chi0: np.ndarray, qpg: np.ndarray) -> np.ndarray:
    """(I - v chi0)^-1 directly: v multiplies chi0 from the left."""
    v = 4.0 * np.pi / np.asarray(qpg, dtype=np.float64) ** 2
    ng = chi0.shape[-1]
    out = np.empty_like(chi0)
    for j in range(chi0.shape[0]):
        out[j] = np.linalg.inv(np.eye(ng) - v[:, None] * chi0[j])
    return out

"""Pins of the plasmon-pole and self-energy oracle (CPU only).

None of these retypes the oracle's formulas: the fit is checked against data made
from known pole parameters, the closed-form correlation self-energy against a
quadrature of the GW product on the imaginary axis, and the exchange against the
Fock sum of free electrons computed without oscillator strengths.
"""

import numpy as np
import pytest
from scipy.integrate import quad

from synth.crystal import sc_lattice, miller_sphere, kgrid_gamma, find_pairs, gset_sorted, qpg_norms
from oracle.rho import rho_direct
from oracle.sigma import ppa_fit, ppa_eval_imag, coulomb_factor, sigma_c_ppa, sigma_x

WP = 1.0
HEAD = 2.5   # stands for the cell average of 4 pi / q^2 at q = 0


def _crand(g, *shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def test_ppa_fit_reproduces_both_samples():
    g = np.random.default_rng(11)
    n = 9
    # a decaying Hermitian response plus noise: most elements valid, some not
    A = _crand(g, n, n) * 0.2
    X0 = -(A @ A.conj().T) - 0.3 * np.eye(n)
    Xp = 0.6 * X0 + 0.05 * _crand(g, n, n)
    R, Om = ppa_fit(X0 + np.eye(n), Xp + np.eye(n), WP)
    d = X0 - Xp
    valid = (Xp.real * d.real + Xp.imag * d.imag) > 0
    assert 0 < valid.sum() < n * n
    assert np.allclose(ppa_eval_imag(R, Om, 0.0), X0, rtol=0, atol=1e-13)
    assert np.allclose(ppa_eval_imag(R, Om, WP)[valid], Xp[valid], rtol=0, atol=1e-13)
    assert np.all(Om.real[valid] > 0)
    assert np.all(Om[~valid] == WP)


@pytest.mark.parametrize("wp", [1.0, 0.7])
def test_ppa_fit_recovers_one_pole_parameters(wp):
    g = np.random.default_rng(5)
    n = 6
    R0 = _crand(g, n, n)
    a = g.uniform(0.3, 2.0, (n, n))
    Om0 = a + 1j * a * g.uniform(-0.9, 0.9, (n, n))      # Re Om^2 > 0
    X0 = -2.0 * R0 / Om0
    Xp = -2.0 * R0 * Om0 / (wp * wp + Om0 * Om0)
    R, Om = ppa_fit(X0 + np.eye(n), Xp + np.eye(n), wp)
    assert np.allclose(Om, Om0, rtol=1e-12, atol=0)
    assert np.allclose(R, R0, rtol=1e-12, atol=0)


def test_sigma_c_equals_imaginary_axis_gw_product():
    # Sigma_c(i nu) = -(1/2pi) int dw sum_m rho rho* W_c(i w) / (i (nu + w) - e_m), energies from
    # the chemical potential (0): occupied bands below it, empty above
    g = np.random.default_rng(3)
    nm, nn, ng = 5, 2, 3
    rho = _crand(g, nm, nn, ng) * 0.5
    e = np.array([-0.9, -0.35, 0.25, 0.8, 1.6])
    f = (e < 0).astype(float)
    Wr = _crand(g, ng, ng)
    a = g.uniform(0.4, 1.5, (ng, ng))
    Om = a + 1j * a * g.uniform(-0.5, 0.5, (ng, ng))
    pref = 0.37
    nus = np.array([[0.3, 1.1], [0.05, 2.0]])
    got = sigma_c_ppa(rho, Wr, Om, e, f, 1j * nus, 0.0, pref)

    for n in range(nn):
        P = [np.outer(rho[m, n], np.conj(rho[m, n])) for m in range(nm)]
        for j in range(2):
            nu = nus[n, j]

            def integrand(w):
                Wc = Wr * (-2.0 * Om / (w * w + Om * Om))
                return -pref / (2 * np.pi) * sum(np.sum(P[m] * Wc) / (1j * (nu + w) - e[m]) for m in range(nm))

            re = quad(lambda w: integrand(w).real, -np.inf, np.inf, epsabs=1e-13, epsrel=1e-12, limit=400)[0]
            im = quad(lambda w: integrand(w).imag, -np.inf, np.inf, epsabs=1e-13, epsrel=1e-12, limit=400)[0]
            ref = re + 1j * im
            assert abs(got[n, j] - ref) <= 1e-9 * max(1.0, abs(ref)), (n, j, got[n, j], ref)


def test_sigma_c_static_sample_of_a_one_pole_response():
    # eps~^-1 at 0 and i omega_p built from known poles; the fitted model gives back the
    # closed form of those poles (every element valid)
    g = np.random.default_rng(8)
    ng = 4
    R0 = _crand(g, ng, ng) * 0.3
    Om0 = g.uniform(0.5, 1.5, (ng, ng)) + 0j
    X0 = -2 * R0 / Om0
    Xp = -2 * R0 * Om0 / (WP ** 2 + Om0 ** 2)
    R, Om = ppa_fit(X0 + np.eye(ng), Xp + np.eye(ng), WP)
    s = g.uniform(0.5, 2.0, ng)
    Wr = R * coulomb_factor(s)
    rho = _crand(g, 2, 1, ng)
    e = np.array([-0.5, 0.7])
    f = np.array([1.0, 0.0])
    z = np.array([[0.1 + 0.0j]])
    got = sigma_c_ppa(rho, Wr, Om, e, f, z, 0.02, 1.0)
    ref = 0.0
    for m in range(2):
        for a in range(ng):
            for b in range(ng):
                w = rho[m, 0, a] * np.conj(rho[m, 0, b]) * R0[a, b] * s[a] * s[b]
                if f[m] > 0:
                    ref += w / (0.1 - e[m] + Om0[a, b] - 0.02j)
                else:
                    ref += w / (0.1 - e[m] - Om0[a, b] + 0.02j)
    assert abs(got[0, 0] - ref) < 1e-12 * abs(ref)


def test_sigma_x_of_plane_waves_is_the_fock_sum():
    # empty lattice: every band is one plane wave, so the exchange of state n is
    # -pref sum over occupied plane waves p_m at every k - q of 4 pi / |p_n - p_m|^2
    lat = sc_lattice(7.0)
    kf = kgrid_gamma(2)
    ecut = 1.2
    mills = [miller_sphere(lat, k, ecut) for k in kf]
    nocc, nstate = 4, 3
    gm = gset_sorted(lat, 400)
    pref = 1.0 / (len(kf) * lat.omega)
    ik0 = 3
    pn = kf[ik0] @ lat.bvec + mills[ik0][:nstate] @ lat.bvec
    sx = np.zeros(nstate)
    direct = np.zeros(nstate)
    for qf in kf:
        pairs = find_pairs(kf, qf)
        _, ikp, g0 = pairs[ik0]
        cn = np.eye(mills[ik0].shape[0], dtype=np.complex128)[:nstate]
        cm = np.eye(mills[ikp].shape[0], dtype=np.complex128)[:nocc + 2]     # two empty bands too
        rho = rho_direct(cn, mills[ik0], cm, mills[ikp], gm, g0)      # [m, n, G]
        s = np.sqrt(4 * np.pi) / qpg_norms(lat, qf, gm)
        q0 = np.all(np.abs(qf) < 1e-12)
        if q0:
            s[0] = 0.0
            # q = 0 with only the head of the Coulomb factor kept: rho_nm(0, 0) = delta_nm, so
            # Sigma_c is the one pole of the head element
            R, Om = np.full((gm.shape[0],) * 2, 0.3 + 0.1j), np.full((gm.shape[0],) * 2, 0.8 + 0.05j)
            Wr = R * coulomb_factor(np.zeros_like(s), HEAD)
            z = np.array([[0.2 + 0.01j]] * nstate)
            sc = sigma_c_ppa(rho[:nocc], Wr, Om, np.zeros(nocc), np.ones(nocc), z, 0.03, pref)
            for n in range(nstate):
                assert abs(sc[n, 0] - pref * HEAD * (0.3 + 0.1j) / (0.2 + 0.01j + 0.8 + 0.05j - 0.03j)) < 1e-14
        sx += sigma_x(rho, np.r_[np.ones(nocc), 0.0, 0.0], s, HEAD if q0 else None, pref)
        pm = kf[ikp] @ lat.bvec + mills[ikp][:nocc] @ lat.bvec
        for n in range(nstate):
            for m in range(nocc):
                d = pn[n] - pm[m]
                dd = d @ d
                direct[n] -= pref * (4 * np.pi / dd if dd > 1e-12 else HEAD)
    # the G-set holds every momentum transfer between the two spheres
    assert np.allclose(sx, direct, rtol=1e-12, atol=0), (sx, direct)
    assert np.all(direct < 0)

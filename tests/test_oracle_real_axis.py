"""Pins of the real-axis response oracle (CPU only).

The real-axis chi0 continues to the imaginary-axis chi0 (itself pinned against
brute force and sum rules) at omega = i w, eta = 0; the spectral weight of every
transition integrates to -pi over omega > 0 for any broadening (this fixes the
placement and sign of both i eta terms); time ordering puts Im chi0_GG below zero
at positive frequencies.
"""

import numpy as np
from scipy.integrate import quad

from synth.rand import random_complex, random_positive
from oracle.chi0 import chi0_from_rho, chi0_real_axis, pole_factor_real_axis


def test_continues_to_the_imaginary_axis():
    M = random_complex(1, (40, 9))
    dE = random_positive(2, 40, 0.1, 2.0)
    ws = [0.0, 0.3, 1.7]
    got = chi0_real_axis(M, dE, [1j * w for w in ws], 0.0, 0.21)
    ref = chi0_from_rho(M, dE, ws, 0.21)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_spectral_weight_integrates_to_minus_pi():
    # B = (chi0 - chi0^H) / 2i = pref sum_t Im F_t rho rho*; int_0^inf Im F_t = -pi for any eta > 0
    M = random_complex(3, (6, 4))
    dE = random_positive(4, 6, 0.2, 1.5)
    pref, eta = 0.5, 0.03
    R = pref * M.T @ np.conj(M)

    def B(w, a, b):
        c = chi0_real_axis(M, dE, [w], eta, pref)[0]
        return (c[a, b] - np.conj(c[b, a])) / 2j

    for a, b in [(0, 0), (1, 3), (2, 1)]:
        parts = []
        for fn in (lambda w: B(w, a, b).real, lambda w: B(w, a, b).imag):
            v = quad(fn, 0, 10, points=list(dE), limit=500, epsabs=1e-13)[0]
            v += quad(fn, 10, np.inf, limit=200, epsabs=1e-13)[0]
            parts.append(v)
        got = parts[0] + 1j * parts[1]
        assert abs(got + np.pi * R[a, b]) <= 1e-7 * np.max(np.abs(R)), (a, b, got, -np.pi * R[a, b])


def test_time_ordering_sign():
    M = random_complex(5, (30, 7))
    dE = random_positive(6, 30, 0.2, 1.5)
    chi = chi0_real_axis(M, dE, [0.1, 0.5, 1.0, 2.5], 0.02, 0.3)
    for c in chi:
        assert np.all(np.diag(c).imag < 0)
    # A and B Hermitian
    A = (chi + np.conj(np.transpose(chi, (0, 2, 1)))) / 2
    B = (chi - np.conj(np.transpose(chi, (0, 2, 1)))) / 2j
    Fs = [pole_factor_real_axis(dE, w, 0.02) for w in [0.1, 0.5, 1.0, 2.5]]
    for j, F in enumerate(Fs):
        assert np.allclose(A[j], 0.3 * (M.T * F.real) @ np.conj(M), rtol=0, atol=1e-12)
        assert np.allclose(B[j], 0.3 * (M.T * F.imag) @ np.conj(M), rtol=0, atol=1e-12)

"""Pins of the oracle trajectory (the toy fluxes of Sec. 2.1's sparse orbit)
against closed forms: the circular inspiral p(t), Phi_phi(t) and plunge time,
Omega_r by quadrature, and the eccentric-orbit invariant."""
import math

import numpy as np
from scipy.integrate import quad

from oracle.trajectory import G_MSUN_OVER_C3, peters_invariant, trajectory


def test_circular_inspiral_closed_form():
    M, mu, p0, T = 1e6, 10.0, 12.0, 1e7
    tr = trajectory(M, mu, p0, 0.0, T, 50)
    Ms, q = M * G_MSUN_OVER_C3, mu / M
    a = 256.0 / 5.0 * q / Ms
    p = (p0 ** 4 - a * tr[0]) ** 0.25
    np.testing.assert_allclose(tr[5], p, rtol=1e-13)
    assert np.all(tr[6] == 0.0)
    phi = 8.0 * (p0 ** 2.5 - p ** 2.5) / (5.0 * a * Ms)
    np.testing.assert_allclose(tr[3][1:], phi[1:], rtol=1e-11)
    np.testing.assert_allclose(tr[1], p ** -1.5 / (2 * math.pi * Ms), rtol=1e-13)
    # Phi_r by quadrature of Omega_r along the closed-form p(t)
    for j in (10, 30, 49):
        val, _ = quad(lambda t: (p0 ** 4 - a * t) ** -0.375 * math.sqrt(1 - 6 * (p0 ** 4 - a * t) ** -0.25) / Ms,
                      0.0, tr[0][j], epsabs=0, epsrel=1e-13, limit=200)
        assert abs(tr[4][j] - val) <= 1e-10 * val


def test_circular_plunge_time():
    M, mu, p0 = 1e5, 50.0, 7.0
    Ms, q = M * G_MSUN_OVER_C3, mu / M
    a = 256.0 / 5.0 * q / Ms
    t_plunge = (p0 ** 4 - 6.1 ** 4) / a
    tr = trajectory(M, mu, p0, 0.0, 10 * t_plunge, 20)
    assert abs(tr[0][-1] - t_plunge) <= 1e-9 * t_plunge
    assert abs(tr[5][-1] - 6.1) <= 1e-10


def test_eccentric_invariant_and_plunge_condition():
    tr = trajectory(1e6, 30.0, 9.5, 0.4, 5e7, 60)
    inv = peters_invariant(tr[5], tr[6])
    assert np.max(np.abs(inv / inv[0] - 1)) <= 1e-12
    assert abs(tr[5][-1] - (6 + 2 * tr[6][-1] + 0.1)) <= 1e-10
    assert tr[0][-1] < 5e7

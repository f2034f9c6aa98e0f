"""Pins of the oracle's spin-weighted spherical harmonics (the angular
functions of Eq. main_wave for a Schwarzschild inspiral)."""
import math

import numpy as np
import pytest

from oracle.harmonics import swsh, swsh_dtheta


@pytest.mark.parametrize("m", list(range(-10, 11)))
def test_orthonormal_gauss_legendre(m):
    """int sY_lm conj(sY_l'm) dOmega = delta_ll' (the integrand is a
    polynomial in cos(theta/2), sin(theta/2) of degree <= 4 lmax, so
    Gauss-Legendre in cos(theta) with enough nodes is exact)."""
    x, wq = np.polynomial.legendre.leggauss(64)
    th = np.arccos(x)
    ls = [l for l in range(2, 11) if abs(m) <= l]
    Y = np.array([swsh(-2, l, m, th, 0.0) for l in ls])
    gram = 2 * math.pi * (Y * wq) @ np.conj(Y).T
    assert np.allclose(gram, np.eye(len(ls)), atol=5e-14, rtol=0)


def test_l2_m2_closed_forms():
    th = np.linspace(0, math.pi, 17)
    ph = 0.37
    c = math.sqrt(5 / (64 * math.pi))
    assert np.allclose(swsh(-2, 2, 2, th, ph), c * (1 + np.cos(th)) ** 2 * np.exp(2j * ph), atol=1e-15)
    assert np.allclose(swsh(-2, 2, -2, th, ph), c * (1 - np.cos(th)) ** 2 * np.exp(-2j * ph), atol=1e-15)


def test_l2_m0_closed_form():
    th = np.linspace(0, math.pi, 17)
    assert np.allclose(swsh(-2, 2, 0, th, 0.0), math.sqrt(15 / (32 * math.pi)) * np.sin(th) ** 2, atol=1e-15)


def test_phi_dependence():
    th = 0.8
    for l, m in [(3, 1), (5, -4), (10, 7)]:
        assert np.allclose(swsh(-2, l, m, th, 0.9), swsh(-2, l, m, th, 0.0) * np.exp(0.9j * m), atol=1e-15)


@pytest.mark.parametrize("lm", [(2, 2), (2, 0), (3, -1), (6, 4), (10, 10), (10, -3)])
def test_dtheta_matches_finite_difference(lm):
    l, m = lm
    th = np.array([0.3, 1.1, 2.0, 2.9])
    h = 1e-6
    fd = (swsh(-2, l, m, th + h, 0.4) - swsh(-2, l, m, th - h, 0.4)) / (2 * h)
    assert np.allclose(swsh_dtheta(-2, l, m, th, 0.4), fd, atol=1e-8, rtol=1e-7)

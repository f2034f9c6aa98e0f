"""Pins of the oracle's per-root SPA factor (Eq. extendedspa1, Sec. 2.2)
against mpmath, the large-argument expansion, symmetry and the standard-SPA
limit the paper states."""
import math

import mpmath
import numpy as np
import pytest

from oracle.special import G, G_airy, G_bessel, W

mpmath.mp.dps = 40


def W_mp(x):
    x = mpmath.mpf(x)
    s = 1 if x > 0 else -1
    return complex(mpmath.sqrt(2 * abs(x) / mpmath.pi) * mpmath.exp(-0.25j * mpmath.pi * s)
                   * mpmath.exp(-1j * x) * mpmath.besselk(mpmath.mpf(1) / 3, -1j * x))


@pytest.mark.parametrize("sign", [1, -1])
def test_W_against_mpmath(sign):
    xs = sign * np.geomspace(1e-6, 1e12, 37)
    got = W(xs)
    for x, g in zip(xs, got):
        ref = W_mp(x)
        assert abs(g - ref) <= 2e-15 * abs(ref), (x, g, ref)


def test_W_large_argument_expansion():
    # DLMF 10.40.2 with nu = 1/3: W = 1 - 5i/(72 X) + O(X^-2)
    for x in [1e3, 1e4, 1e5, 1e6]:
        w = complex(W(np.array([x]))[0])
        assert abs(w - (1 - 5j / (72 * x))) <= 0.05 / x ** 2


def test_W_conjugate_symmetry():
    xs = np.geomspace(1e-5, 1e9, 29)
    assert np.allclose(W(-xs), np.conj(W(xs)), rtol=1e-15, atol=0)


def test_W_small_argument_limit():
    # K_{1/3}(z) ~ Gamma(1/3)/2 (z/2)^{-1/3}: W ~ sqrt(2X/pi) Gamma(1/3)/2 (X/2)^{-1/3} e^{-i pi/4} e^{i pi/6}
    x = 1e-9
    ref = (math.sqrt(2 * x / math.pi) * math.gamma(1 / 3) / 2 * (x / 2) ** (-1 / 3)
           * np.exp(-0.25j * math.pi) * np.exp(1j * math.pi / 6))
    assert abs(W(np.array([x]))[0] - ref) <= 1e-5 * abs(ref)


@pytest.mark.parametrize("X", [0.05, 0.3, 0.9, 1.1, 2.0, 5.0])
@pytest.mark.parametrize("sign", [1, -1])
def test_airy_and_bessel_forms_agree(X, sign):
    Fdd = 3e-17
    Fd = sign * (X * 3 * Fdd ** 2 / (2 * math.pi)) ** (1 / 3)
    ga = G_airy(np.array([Fd]), np.array([Fdd]), np.array([sign]))[0]
    gb = G_bessel(np.array([Fd]), np.array([Fdd]))[0]
    assert abs(ga - gb) <= 3e-15 * abs(gb)


@pytest.mark.parametrize("Fd", [3e-12, -3e-12])
def test_standard_spa_limit(Fd):
    """Fdd -> 0 must give the standard SPA factor 1/sqrt(i Fd) (the paper's
    statement after Eq. extendedspa1)."""
    spa = abs(Fd) ** -0.5 * np.exp(-0.25j * math.pi * np.sign(Fd))
    for Fdd in [1e-22, 1e-24, 1e-28, 0.0]:
        g = G(np.array([Fd]), np.array([Fdd]), np.sign(Fd))[0]
        X = 2 * math.pi * Fd ** 3 / (3 * Fdd ** 2) if Fdd else math.inf
        assert abs(g - spa) <= (0.08 / abs(X) + 1e-15) * abs(spa)


def test_printed_constant_is_minus_G():
    """Eq. extendedspa1 as printed, (2/sqrt3)(i Fd/|Fdd|) e^{-iX} K_{1/3}(-iX),
    on the principal branch is exactly -G: the reading that flips its sign."""
    for Fd, Fdd in [(2e-12, 1e-18), (-2e-12, 1e-18), (5e-13, -4e-19), (-1e-12, -1e-17)]:
        X = mpmath.mpf(2) * mpmath.pi * mpmath.mpf(Fd) ** 3 / (3 * mpmath.mpf(Fdd) ** 2)
        lit = (2 / mpmath.sqrt(3)) * (1j * mpmath.mpf(Fd) / abs(mpmath.mpf(Fdd))) \
            * mpmath.exp(-1j * X) * mpmath.besselk(mpmath.mpf(1) / 3, -1j * X)
        g = G(np.array([Fd]), np.array([Fdd]), np.sign(Fd))[0]
        assert abs(g + complex(lit)) <= 1e-14 * abs(g)


def test_turnover_value_finite_and_directional():
    """At Fd = 0 the factor is finite; the two sides are conjugate."""
    gp = G(np.array([0.0]), np.array([2e-18]), 1.0)[0]
    gm = G(np.array([0.0]), np.array([2e-18]), -1.0)[0]
    c = math.pi * (math.pi * 2e-18) ** (-1 / 3)
    ai0, bi0 = float(mpmath.airyai(0)), float(mpmath.airybi(0))
    assert abs(gp - c * (ai0 - 1j * bi0)) <= 1e-14 * abs(gp)
    assert abs(gm - np.conj(gp)) <= 1e-15 * abs(gp)
    assert G(np.array([0.0]), np.array([0.0]), 1.0)[0] == 0


def test_iintegral_identity_for_real_alpha():
    """Eq. Iintegral for real alpha > 0, by direct quadrature."""
    for alpha, beta in [(1.0, 0.5), (0.7, -1.3), (2.0, 3.0)]:
        a, b = mpmath.mpf(alpha), mpmath.mpf(beta)
        lhs = mpmath.quad(lambda t: mpmath.exp(-a * t * t / 2 - 1j * b * t ** 3 / 6), [-mpmath.inf, 0, mpmath.inf])
        z = a ** 3 / (3 * b * b)
        rhs = 2 / mpmath.sqrt(3) * a / abs(b) * mpmath.exp(z) * mpmath.besselk(mpmath.mpf(1) / 3, z)
        assert abs(lhs - rhs) <= 1e-6 * abs(rhs)   # quadrature of an oscillatory tail

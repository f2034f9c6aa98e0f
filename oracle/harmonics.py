"""Spin-weighted spherical harmonics sY_lm(theta, phi) (oracle, test
infrastructure).

For a Schwarzschild inspiral the angular functions S_lmkn of Eq. main_wave
are the spin-weighted spherical harmonics with s = -2 (Sec. 2.1); together
with the e^{i m phi} factor of that equation they form sY_lm(theta, phi).
Written here from the Goldberg explicit sum:

  sY_lm = (-1)^m sqrt[(l+m)!(l-m)!(2l+1) / (4 pi (l+s)!(l-s)!)]
          * sum_r C(l-s, r) C(l+s, r+s-m) (-1)^(l-r-s)
            * sin(theta/2)^(2l-k) cos(theta/2)^k e^{i m phi},  k = 2r+s-m,

i.e. sin^{2l}(theta/2) cot^k(theta/2) expanded so that theta = 0, pi need no
division.  Pinned by orthonormality under Gauss-Legendre quadrature and by
the closed forms of -2Y_{2,+-2}.
"""
from __future__ import annotations

import math

import numpy as np


def _terms(s: int, l: int, m: int):
    if l < abs(s) or abs(m) > l:
        raise ValueError(f"invalid (s,l,m)=({s},{l},{m})")
    pref = (-1) ** m * math.sqrt(math.factorial(l + m) * math.factorial(l - m) * (2 * l + 1)
                                 / (4 * math.pi * math.factorial(l + s) * math.factorial(l - s)))
    out = []
    for r in range(0, l - s + 1):
        b2 = r + s - m
        if b2 < 0 or b2 > l + s:
            continue
        c = math.comb(l - s, r) * math.comb(l + s, b2) * (-1) ** (l - r - s)
        k = 2 * r + s - m
        out.append((pref * c, k))
    return out


def swsh(s: int, l: int, m: int, theta, phi):
    """sY_lm(theta, phi) in FP64 (complex)."""
    theta = np.asarray(theta, np.float64)
    ch, sh = np.cos(theta / 2), np.sin(theta / 2)
    acc = np.zeros(np.broadcast(theta, phi).shape, np.float64)
    for c, k in _terms(s, l, m):
        acc = acc + c * sh ** (2 * l - k) * ch ** k
    return acc * np.exp(1j * m * np.asarray(phi, np.float64))


def swsh_dtheta(s: int, l: int, m: int, theta, phi):
    """d/dtheta of sY_lm, differentiating each term of the same sum:
    d/dtheta [sh^a ch^k] = (a ch^2 - k sh^2) sh^(a-1) ch^(k-1) / 2."""
    theta = np.asarray(theta, np.float64)
    ch, sh = np.cos(theta / 2), np.sin(theta / 2)
    acc = np.zeros(np.broadcast(theta, phi).shape, np.float64)
    for c, k in _terms(s, l, m):
        a = 2 * l - k
        term = 0.0
        if a > 0:
            term = term + 0.5 * a * sh ** (a - 1) * ch ** (k + 1)
        if k > 0:
            term = term - 0.5 * k * sh ** (a + 1) * ch ** (k - 1)
        acc = acc + c * term
    return acc * np.exp(1j * m * np.asarray(phi, np.float64))

"""Per-root third-order stationary-phase factor (oracle, test infrastructure).

Eq. extendedspa1 gives, for each root t_j of F(t) = f with local
derivatives Fd = dF/dt and Fdd = d^2F/dt^2 there, the factor multiplying
H(t_j) e^{i[2 pi f t_j - Phi(t_j)]}:

  G = c (i Fd / |Fdd|) e^{-i X} K_{1/3}(-i X),   X = 2 pi Fd^3 / (3 Fdd^2).

Readings used here (each justified in the design notes):
  * X is real (the stray i in its definition after Eq. extendedspa1 is
    dropped); the special function is taken on the principal branch.
  * The overall constant is c = -2/sqrt(3): with the printed +2/sqrt(3) the
    formula tends to minus the standard SPA as Fdd -> 0, contradicting the
    paper's own statement that it reduces to the standard SPA in that limit.
    With -2/sqrt(3) it equals

      G = |Fd|^{-1/2} e^{-i pi/4 sgn Fd} W(X),
      W(X) = sqrt(2|X|/pi) e^{-i pi/4 sgn X} e^{-iX} K_{1/3}(-iX),

    W -> 1 as |X| -> inf (standard SPA), W(-X) = conj W(X).
  * Fdd = 0 exactly: W = 1 (standard SPA).
  * Small |X| (near a frequency turnover, Fd -> 0) the same factor is written
    with Airy functions, which stays finite at Fd = 0:

      G = pi (pi |Fdd|)^{-1/3} [Ai(-zeta) - i s Bi(-zeta)] e^{-i s |X|},
      zeta = (3|X|/2)^{2/3} = pi^{2/3} Fd^2 / |Fdd|^{4/3},  s = sgn Fd,

    with s taken as the direction of the monotonic piece the root belongs to
    when Fd = 0 exactly.
  * Fd = Fdd = 0 (a flat inflection, outside the method): contributes 0.

W uses scipy's exponentially scaled K (kve) for |X| <= 1e4 and the
large-argument expansion W = sum_k a_k (i/X)^k,
a_k = prod_{j<=k} (4 nu^2 - (2j-1)^2) / (k! 8^k), nu = 1/3, beyond.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import airy, kve

NU = 1.0 / 3.0
X_AIRY = 1.0        # |X| below this: Airy form
X_ASYMP = 1e4       # |X| above this: large-argument expansion (8 terms)


def _asymp_coeffs(nterms: int):
    a = [1.0]
    for k in range(1, nterms):
        a.append(a[-1] * (4 * NU * NU - (2 * k - 1) ** 2) / (k * 8.0))
    return a


_ASYMP = _asymp_coeffs(8)


def W(X):
    """Normalised special function W(X) for real X != 0 (complex128)."""
    X = np.asarray(X, np.float64)
    out = np.empty(X.shape, np.complex128)
    ax = np.abs(X)
    big = ax > X_ASYMP
    mid = ~big
    if np.any(mid):
        x = X[mid]
        pref = np.sqrt(2.0 * np.abs(x) / math.pi) * np.exp(-0.25j * math.pi * np.sign(x))
        out[mid] = pref * kve(NU, -1j * x)
    if np.any(big):
        u = 1j / X[big]
        acc = np.zeros(u.shape, np.complex128)
        for a in reversed(_ASYMP):
            acc = acc * u + a
        out[big] = acc
    return out


def G_bessel(Fd, Fdd):
    """G through W(X); requires Fd != 0."""
    Fd = np.asarray(Fd, np.float64)
    Fdd = np.asarray(Fdd, np.float64)
    sgn = np.sign(Fd)
    base = np.abs(Fd) ** -0.5 * np.exp(-0.25j * math.pi * sgn)
    out = base.astype(np.complex128)
    nz = Fdd != 0
    if np.any(nz):
        r = Fd[nz] / Fdd[nz]
        X = (2.0 * math.pi / 3.0) * Fd[nz] * r * r
        out[nz] = base[nz] * W(X)
    return out


def G_airy(Fd, Fdd, s):
    """G through Airy functions; requires Fdd != 0.  s = +-1 is sgn Fd (or
    the piece direction when Fd = 0)."""
    Fd = np.asarray(Fd, np.float64)
    Fdd = np.asarray(Fdd, np.float64)
    s = np.asarray(s, np.float64)
    c = (math.pi * np.abs(Fdd)) ** (-1.0 / 3.0)
    y = math.pi ** (1.0 / 3.0) * np.abs(Fd) / np.abs(Fdd) ** (2.0 / 3.0)
    zeta = y * y
    ax = (2.0 / 3.0) * y ** 3
    ai, _, bi, _ = airy(-zeta)
    return math.pi * c * (ai - 1j * s * bi) * np.exp(-1j * s * ax)


def G(Fd, Fdd, direction):
    """Per-root factor of Eq. extendedspa1 (with the readings above).
    direction = +-1 is the sign of dF/dt on the root's monotonic piece."""
    Fd = np.atleast_1d(np.asarray(Fd, np.float64))
    Fdd = np.atleast_1d(np.asarray(Fdd, np.float64))
    direction = np.broadcast_to(np.asarray(direction, np.float64), Fd.shape)
    out = np.zeros(Fd.shape, np.complex128)
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        r = Fd / Fdd
        X = (2.0 * math.pi / 3.0) * Fd * r * r
    flat = (Fd == 0) & (Fdd == 0)
    spa = (Fdd == 0) & ~flat
    airy_m = (Fdd != 0) & (np.abs(X) < X_AIRY)
    bes = ~flat & ~spa & ~airy_m
    if np.any(spa | bes):
        idx = spa | bes
        out[idx] = G_bessel(Fd[idx], Fdd[idx])
    if np.any(airy_m):
        s = np.where(Fd[airy_m] != 0, np.sign(Fd[airy_m]), direction[airy_m])
        out[airy_m] = G_airy(Fd[airy_m], Fdd[airy_m], s)
    return out

"""Inner product and Whittle log-likelihood (oracle, test infrastructure).

Eq. innerprod:   <a|b> = 4 Re sum_k conj(a_k) b_k / S(f_k) * w_k,
with w_k = 1/T on the DFT grid f_k = k/T (k >= 1); on other grids the
trapezoid weights of the grid are used (the continuous integral of
Eq. innerprod).  The DC bin (f = 0) is excluded.

Eq. likelihood:  log p = -1/2 sum_{alpha=+,x} <d - h | d - h>_alpha.

fused_sums gives the three sums of the fused likelihood (fdemri_loglike) by
their definitions, with the per-bin weight wS_k = 4 w_k / S(f_k) taken as an
input.
"""
from __future__ import annotations

import numpy as np


def grid_weights(f):
    """Quadrature weights of the frequency grid: 1/T = f_1 - f_0 on a uniform
    grid, trapezoid weights otherwise; zero for f = 0."""
    f = np.asarray(f, np.float64)
    w = np.zeros(f.size)
    if f.size == 1:
        w[:] = 1.0
    else:
        df = np.diff(f)
        if np.allclose(df, df[0], rtol=1e-9, atol=0):
            w[:] = df[0]
        else:
            w[:-1] += 0.5 * df
            w[1:] += 0.5 * df
    w[f == 0] = 0.0
    return w


def inner_product(a, b, S, w):
    S = np.asarray(S, np.float64)
    good = np.isfinite(S) & (w > 0)
    return 4.0 * np.real(np.sum(np.conj(a[good]) * b[good] / S[good] * w[good]))


def whittle_loglike(d, h, S, w):
    """d, h: (h_plus, h_cross) pairs."""
    return -0.5 * sum(inner_product(di - hi, di - hi, S, w) for di, hi in zip(d, h))


def fused_sums(d, h, wS, hann=False):
    """(log L, <h|h>, <d|h>) over the two channels for data d = (d_+, d_x) and
    model h = (h_+, h_x), each bin weighted by wS:
        log L = -1/2 sum_alpha sum_k wS_k |d_k - g_k|^2,
        <h|h> = sum_alpha sum_k wS_k |g_k|^2,
        <d|h> = sum_alpha sum_k wS_k Re(conj(d_k) g_k),
    with g = fd_hann(h) (the frequency-domain Hann window of the DFT grid)
    when hann, else g = h."""
    from .td import fd_hann
    wS = np.asarray(wS, np.float64)
    ll = hh = dh = 0.0
    for da, ha in zip(d, h):
        g = fd_hann(np.asarray(ha, np.complex128)) if hann else np.asarray(ha, np.complex128)
        da = np.asarray(da, np.complex128)
        ll += -0.5 * float(np.sum(wS * np.abs(da - g) ** 2))
        hh += float(np.sum(wS * np.abs(g) ** 2))
        dh += float(np.sum(wS * np.real(np.conj(da) * g)))
    return ll, hh, dh

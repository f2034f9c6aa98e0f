"""Gradient of a real loss of the waveform (oracle, test infrastructure).

For a loss L(h_+, h_x) with cotangents g_alpha = dL/dRe h_alpha + i dL/dIm h_alpha
(for the Whittle log-likelihood of Eq. likelihood, g = 4 w (d - h) / S), the
explicit-voice sum of oracle.waveform gives the gradient term by term:

  h_+ = [h(f) + conj h(-f)]/2,  h_x = i [h(f) - conj h(-f)]/2 (Eq. main_wave)
  => dL = Re(conj(G+) dh(f)) + Re(conj(G-) dh(-f)),
     G+ = (g_+ - i g_x)/2,  G- = (conj g_+ - i conj g_x)/2.

Each root term T = factor * A(t_j)^(conj) * e^{i psi} G_j (Eq. extendedspa1)
depends on
  * the amplitude spline coefficients a_k of its segment through
    A = sum_k a_k tau^k (holomorphically, or anti-holomorphically for the
    partner voice, which carries conj A);
  * the phase spline coefficients through psi = 2 pi f t - (m Phi_phi + n Phi_r),
    d psi / d c^phi_k = -m tau^k (and -n tau^k for Phi_r);
  * theta, phi, scale through factor = scale Y_{l,m}(theta, phi);
  * Phi_phi0, Phi_r0 as the constant coefficient of every segment.
The root times t_j depend only on the frequency splines, which are held
fixed.  Complex gradients use the same convention dL/dRe + i dL/dIm.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline

from .harmonics import swsh, swsh_dtheta
from .likelihood import grid_weights
from .waveform import Voice, root_terms, splines, waveform_voices


def _voices_with_derivs(l, m, n, theta, phi, scale, partners=True):
    """Explicit voices plus d(factor)/d theta for each."""
    out = []
    for mu, (li, mi, ni) in enumerate(zip(np.asarray(l), np.asarray(m), np.asarray(n))):
        li, mi, ni = int(li), int(mi), int(ni)
        y = complex(swsh(-2, li, mi, theta, phi))
        dy = complex(swsh_dtheta(-2, li, mi, theta, phi))
        out.append((Voice(mi, ni, mu, False, scale * y), scale * dy))
        if partners and mi > 0:
            sg = (-1) ** li
            yp = complex(swsh(-2, li, -mi, theta, phi))
            dyp = complex(swsh_dtheta(-2, li, -mi, theta, phi))
            out.append((Voice(-mi, -ni, mu, True, scale * sg * yp), scale * sg * dyp))
    return out


def waveform_vjp(w, g_p, g_c, f=None, partners=True):
    """Gradients of L with respect to the amplitude and phase spline
    coefficients (ascending powers) and the scalars, for cotangents g_p, g_c
    on the grid f.  Returns dict(gA [Nm, K-1, 4] complex, gPhi [2, K-1, 4],
    g_scalars [5]: theta, phi, scale, Phi_phi0, Phi_r0)."""
    f = w.f if f is None else np.asarray(f)
    sp = splines(w.traj, w.A)
    K = w.traj.t.size
    Gpos = 0.5 * (np.asarray(g_p) - 1j * np.asarray(g_c))
    Gneg = 0.5 * (np.conj(g_p) - 1j * np.conj(g_c))
    gA = np.zeros((w.Nm, K - 1, 4), np.complex128)
    gPhi = np.zeros((2, K - 1, 4))
    g_th = g_ph = g_sc = 0.0
    for v, dfac_dth in _voices_with_derivs(w.l, w.m, w.n, w.theta, w.phi, w.scale, partners):
        for s, k, seg, tau, amp, E in root_terms(w.traj, sp, v, f):
            Gs = Gpos[k] if s > 0 else Gneg[k]
            ampc = np.conj(amp) if v.conj else amp
            T = v.factor * ampc * E
            powers = np.stack([np.ones_like(tau), tau, tau * tau, tau * tau * tau])
            for kp in range(4):
                D = v.factor * powers[kp] * E
                contrib = (np.conj(Gs) * D) if v.conj else (Gs * np.conj(D))
                np.add.at(gA[:, :, kp], (np.full(seg.size, v.mode), seg), contrib)
                im = np.imag(np.conj(Gs) * T) * powers[kp]
                np.add.at(gPhi[0, :, kp], seg, v.m * im)
                np.add.at(gPhi[1, :, kp], seg, v.n * im)
            g_sc += float(np.sum(np.real(np.conj(Gs) * T))) / w.scale
            g_th += float(np.sum(np.real(np.conj(Gs) * dfac_dth * ampc * E)))
            g_ph += float(np.sum(np.real(np.conj(Gs) * 1j * v.m * T)))
    g_scalars = np.array([g_th, g_ph, g_sc, gPhi[0, :, 0].sum(), gPhi[1, :, 0].sum()])
    return dict(gA=gA, gPhi=gPhi, g_scalars=g_scalars)


def whittle_cotangent(d, h, S, wts):
    """g_alpha = dL/dRe h + i dL/dIm h of L = -1/2 sum_alpha <d-h|d-h>_alpha."""
    good = np.isfinite(S) & (wts > 0)
    out = []
    for da, ha in zip(d, h):
        g = np.zeros(ha.shape, np.complex128)
        g[good] = 4.0 * wts[good] * (da[good] - ha[good]) / S[good]
        out.append(g)
    return out


def loglike_and_grad(w, d, S, wts=None, partners=True):
    """Whittle log-likelihood of the data d = (d_+, d_x) for the waveform of w
    (Eq. likelihood with Eq. innerprod) and its gradient (waveform_vjp)."""
    from .likelihood import whittle_loglike
    wts = grid_weights(w.f) if wts is None else wts
    sp = splines(w.traj, w.A)
    from .waveform import voices_from_modes
    h = waveform_voices(w.traj, sp, voices_from_modes(w.l, w.m, w.n, w.theta, w.phi, w.scale, partners), w.f)
    L = whittle_loglike(d, h, S, wts)
    g_p, g_c = whittle_cotangent(d, h, S, wts)
    return L, waveform_vjp(w, g_p, g_c, partners=partners)


def spline_matrix(t):
    """The linear map knot values -> not-a-knot coefficients (ascending
    powers), as an array M[K-1, 4, K] with c[i, k] = sum_j M[i, k, j] y_j,
    built by splining the unit vectors with scipy's CubicSpline."""
    K = t.size
    c = CubicSpline(t, np.eye(K)).c          # (4, K-1, K), highest power first
    return np.transpose(c[::-1], (1, 0, 2))


def coef_grad_to_knots(t, g_coef):
    """Gradient w.r.t. knot values from the gradient w.r.t. coefficients
    (..., K-1, 4) -> (..., K), by the transpose of spline_matrix."""
    M = spline_matrix(t)
    return np.einsum("...ik,ikj->...j", g_coef, M)

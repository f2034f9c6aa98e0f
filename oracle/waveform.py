"""Frequency-domain EMRI waveform by the extended SPA (oracle, test
infrastructure).

Steps, in the order of the method (Sec. 2.1-2.2):

O1  Not-a-knot cubic splines in t of the fundamental frequencies F_phi, F_r,
    the phases Phi_phi, Phi_r and the complex mode amplitudes A_lmn
    (Sec. 2.1: amplitudes and phases; Sec. 2.2: frequencies).  scipy's
    CubicSpline (default not-a-knot) serves as the library primitive.
O2  Explicit voices (Eq. wave_voice): for every (l,m,n) of the table the
    voice V with H_V = scale A Y_lm(theta, phi), Phi_V = m Phi_phi + n Phi_r,
    F_V = m F_phi + n F_r (Eq. main_wave, k = 0).  For m > 0 also the voice
    (l,-m,-n) with H = scale (-1)^l conj(A) Y_{l,-m}, Phi = -Phi_V, F = -F_V;
    m = 0 entries are their own partners' table rows.
O3  For every voice and every grid frequency f > 0, all times with
    F_V(t) = +f (they feed h(+f)) and F_V(t) = -f (they feed h(-f)).  The
    spline of F_V is the cubic of Eq. cubic_equation on each segment; it is
    split into monotonic pieces at the zeros of dF_V/dt and of F_V, and the
    unique root in each piece is found by bisection to full FP64 precision.
    Piece end values at knots use the knot data m F_phi,i + n F_r,i.
O4  dF/dt and d^2F/dt^2 at the root from the frequency spline (Sec. 2.2).
O5  The per-root factor G of Eq. extendedspa1 (see oracle.special).
O6  h(sigma f) = sum_V sum_j H_V(t_j) e^{i[2 pi sigma f t_j - Phi_V(t_j)]} G_j
    (Eqs. SPAintegral2, extendedspa1), with the large phase formed in
    extended precision and reduced modulo 2 pi before the sine/cosine.
O7  h = h_+ - i h_x (Eq. main_wave) with the transform convention of
    Eq. singlevoiceFT gives
      h_+(f) = [h(f) + conj h(-f)] / 2,  h_x(f) = i [h(f) - conj h(-f)] / 2,
    and 0 at f = 0.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np
from scipy.interpolate import CubicSpline, PPoly

from .harmonics import swsh
from .special import G

TWO_PI_LD = np.longdouble("6.283185307179586476925286766559005768394")


@dataclass
class Voice:
    m: int              # F_V = m F_phi + n F_r, Phi_V = m Phi_phi + n Phi_r
    n: int
    mode: int           # row of the amplitude table
    conj: bool          # amplitude enters as conj(A)
    factor: complex     # multiplies A or conj(A)


def splines(traj, A):
    """O1: scipy not-a-knot coefficient arrays, highest power first:
    c[0] tau^3 + c[1] tau^2 + c[2] tau + c[3] on [t_i, t_{i+1}]."""
    t = traj.t
    out = {}
    for key in ("Fphi", "Fr", "Phiphi", "Phir"):
        out[key] = CubicSpline(t, getattr(traj, key)).c
    out["A"] = CubicSpline(t, np.asarray(A).T).c     # (4, K-1, Nm) complex
    return out


def voices_from_modes(l, m, n, theta, phi, scale, partners=True):
    """O2: explicit voice list for an m >= 0 mode table."""
    vs = []
    for mu, (li, mi, ni) in enumerate(zip(np.asarray(l), np.asarray(m), np.asarray(n))):
        li, mi, ni = int(li), int(mi), int(ni)
        y = complex(swsh(-2, li, mi, theta, phi))
        vs.append(Voice(mi, ni, mu, False, scale * y))
        if partners and mi > 0:
            yp = complex(swsh(-2, li, -mi, theta, phi))
            vs.append(Voice(-mi, -ni, mu, True, scale * (-1) ** li * yp))
    return vs


def _horner(c, tau):
    """c: (4, ...) highest power first."""
    return ((c[0] * tau + c[1]) * tau + c[2]) * tau + c[3]


def voice_pieces(t, cF, knotF):
    """O3: monotonic pieces of the frequency spline of one voice.

    Returns a list of (ta, tb, Fa, Fb): piece end times and the frequency at
    each end (knot data at the trajectory ends, 0 at zero crossings, the
    spline value at turning points)."""
    pp = PPoly(cF, t)
    t0, t1 = t[0], t[-1]
    tp = pp.derivative().roots(extrapolate=False)
    zc = pp.roots(extrapolate=False)
    tol = 1e-12 * (t1 - t0)
    cand = [(float(x), "turn") for x in tp if np.isfinite(x) and t0 + tol < x < t1 - tol]
    cand += [(float(x), "zero") for x in zc if np.isfinite(x) and t0 + tol < x < t1 - tol]
    cand.sort()
    bps = [(float(t0), "knot0")]
    for x, kind in cand:
        if x - bps[-1][0] <= tol:
            if kind == "zero":
                bps[-1] = (bps[-1][0], "zero") if bps[-1][1] != "knot0" else bps[-1]
            continue
        bps.append((x, kind))
    if t1 - bps[-1][0] <= tol and len(bps) > 1:
        bps.pop()
    bps.append((float(t1), "knotN"))

    def fval(x, kind):
        if kind == "knot0":
            return float(knotF[0])
        if kind == "knotN":
            return float(knotF[-1])
        if kind == "zero":
            return 0.0
        return float(pp(x))

    pieces = []
    for (ta, ka), (tb, kb) in zip(bps[:-1], bps[1:]):
        Fa, Fb = fval(ta, ka), fval(tb, kb)
        if Fa == Fb:
            continue
        pieces.append((ta, tb, Fa, Fb))
    return pieces


def _roots_in_piece(t, cF, knotF, ta, tb, Fa, Fb, y):
    """Times in [ta, tb] where the (monotonic) spline equals y (array), by
    locating the spline segment and bisecting on its cubic.  Returns the
    segment index and tau = t - t_seg for each y."""
    inner = np.nonzero((t > ta) & (t < tb))[0]
    sub_t = np.concatenate(([ta], t[inner], [tb]))
    sub_F = np.concatenate(([Fa], knotF[inner], [Fb]))
    d = 1.0 if Fb > Fa else -1.0
    # sub-interval j with y between sub_F[j] and sub_F[j+1] (lower one on ties)
    j = np.searchsorted(d * sub_F, d * y, side="left") - 1
    j = np.clip(j, 0, sub_t.size - 2)
    a_t, b_t = sub_t[j], sub_t[j + 1]
    seg = np.clip(np.searchsorted(t, a_t, side="right") - 1, 0, t.size - 2)
    c = cF[:, seg]
    lo = a_t - t[seg]
    hi = b_t - t[seg]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        done = (mid == lo) | (mid == hi)
        if np.all(done):
            break
        below = d * (_horner(c, mid) - y) < 0      # root lies above mid
        lo = np.where(below & ~done, mid, lo)
        hi = np.where(~below & ~done, mid, hi)
    return seg, 0.5 * (lo + hi)


def root_terms(traj, sp, v, f):
    """O3-O6 for one voice: yields, for each monotonic piece, the side s
    (+1: the terms feed h(+f); -1: h(-f)), the bin indices k, the spline
    segment and tau of each root, the amplitude spline value A(t_j) (before
    conjugation) and E = e^{i psi} G, so that the voice adds
    factor * (A or conj A) * E to h(s f_k)."""
    t = traj.t
    f = np.asarray(f, np.float64)
    pos_f = f > 0
    cF = v.m * sp["Fphi"] + v.n * sp["Fr"]
    knotF = v.m * traj.Fphi + v.n * traj.Fr
    cPphi = sp["Phiphi"].astype(np.longdouble)
    cPr = sp["Phir"].astype(np.longdouble)
    t_ld = t.astype(np.longdouble)
    for ta, tb, Fa, Fb in voice_pieces(t, cF, knotF):
        lo_F, hi_F = min(Fa, Fb), max(Fa, Fb)
        s = 1.0 if (Fa + Fb) > 0 else -1.0        # sign of F_V on the piece
        dirV = 1.0 if Fb > Fa else -1.0          # direction of F_V on the piece
        k = np.nonzero(pos_f & (s * f >= lo_F) & (s * f <= hi_F))[0]
        if k.size == 0:
            continue
        y = s * f[k]
        seg, tau = _roots_in_piece(t, cF, knotF, ta, tb, Fa, Fb, y)
        c = cF[:, seg]
        Fd = (3.0 * c[0] * tau + 2.0 * c[1]) * tau + c[2]
        Fdd = 6.0 * c[0] * tau + 2.0 * c[1]
        Gj = G(Fd, Fdd, dirV)
        # O6 phase in extended precision
        tau_ld = tau.astype(np.longdouble)
        phiV = (v.m * _horner(cPphi[:, seg], tau_ld) + v.n * _horner(cPr[:, seg], tau_ld))
        psi = TWO_PI_LD * y.astype(np.longdouble) * (t_ld[seg] + tau_ld) - phiV
        psi = psi - TWO_PI_LD * np.round(psi / TWO_PI_LD)
        psi = psi.astype(np.float64)
        amp = _horner(sp["A"][:, seg, v.mode], tau)
        E = (np.cos(psi) + 1j * np.sin(psi)) * Gj
        yield s, k, seg, tau, amp, E


def waveform_voices(traj, sp, voices, f, return_sides=False):
    """O3-O7 for an explicit voice list.  Returns (h_plus, h_cross) on f."""
    f = np.asarray(f, np.float64)
    hpos = np.zeros(f.size, np.complex128)
    hneg = np.zeros(f.size, np.complex128)
    for v in voices:
        for s, k, seg, tau, amp, E in root_terms(traj, sp, v, f):
            term = v.factor * (np.conj(amp) if v.conj else amp) * E
            np.add.at(hpos if s > 0 else hneg, k, term)
    hp = 0.5 * (hpos + np.conj(hneg))
    hc = 0.5j * (hpos - np.conj(hneg))
    pos_f = f > 0
    hp[~pos_f] = 0
    hc[~pos_f] = 0
    if return_sides:
        return hp, hc, hpos, hneg
    return hp, hc


def waveform(w, f=None, partners=True, return_sides=False):
    """Oracle waveform for a workloads.Workload: (h_plus, h_cross) complex128."""
    sp = splines(w.traj, w.A)
    vs = voices_from_modes(w.l, w.m, w.n, w.theta, w.phi, w.scale, partners)
    return waveform_voices(w.traj, sp, vs, w.f if f is None else f, return_sides)


def count_evals(w, f=None):
    """Number of (monotonic piece of |F_V|, bin) pairs for the m >= 0 table:
    the unit of work of the mode sum."""
    f = w.f if f is None else f
    sp = splines(w.traj, w.A)
    total = 0
    for mi, ni in zip(w.m, w.n):
        cF = int(mi) * sp["Fphi"] + int(ni) * sp["Fr"]
        knotF = int(mi) * w.traj.Fphi + int(ni) * w.traj.Fr
        for ta, tb, Fa, Fb in voice_pieces(w.traj.t, cF, knotF):
            lo, hi = sorted((abs(Fa), abs(Fb)))
            total += int(np.count_nonzero((f > 0) & (f >= lo) & (f <= hi)))
    return total

"""Time-domain voice sum and its windowed DFT (oracle, test infrastructure).

Used only to pin the frequency-domain oracle against a true Fourier
transform (Sec. 2.3): h(t) = sum_V H_V(t) e^{-i Phi_V(t)} (Eq. wave_voice)
from the same splines, h_+ = Re h, h_x = -Im h (Eq. main_wave), a Hann window
in the time domain and the matching three-tap convolution in the frequency
domain, and the transform sign of Eq. singlevoiceFT.
"""
from __future__ import annotations

import numpy as np

from .waveform import splines, voices_from_modes, _horner


def td_waveform(w, t_samples, partners=True):
    """Complex h(t_k) on the given sample times (0 outside the trajectory)."""
    sp = splines(w.traj, w.A)
    t = w.traj.t
    ts = np.asarray(t_samples, np.float64)
    inside = (ts >= t[0]) & (ts <= t[-1])
    seg = np.clip(np.searchsorted(t, ts, side="right") - 1, 0, t.size - 2)
    tau = ts - t[seg]
    h = np.zeros(ts.size, np.complex128)
    Pphi = _horner(sp["Phiphi"][:, seg], tau)
    Pr = _horner(sp["Phir"][:, seg], tau)
    for v in voices_from_modes(w.l, w.m, w.n, w.theta, w.phi, w.scale, partners):
        amp = _horner(sp["A"][:, seg, v.mode], tau)
        if v.conj:
            amp = np.conj(amp)
        h += v.factor * amp * np.exp(-1j * (v.m * Pphi + v.n * Pr))
    h[~inside] = 0
    return h


def hann(N):
    k = np.arange(N)
    return 0.5 - 0.5 * np.cos(2 * np.pi * k / N)


def td_spectrum(x_real, dt, window=True):
    """x~(f_k) = dt * conj(rfft(x w))[k] for a real series (e^{+2 pi i f t})."""
    x = np.asarray(x_real, np.float64)
    if window:
        x = x * hann(x.size)
    return dt * np.conj(np.fft.rfft(x))


def fd_hann(h):
    """Frequency-domain Hann window on the DFT grid:
    h_w(f_k) = h(f_k)/2 - h(f_{k+1})/4 - h(f_{k-1})/4, using
    h(-f_1) = conj h(f_1) for the transform of a real series at k = 0 and
    dropping the missing neighbour at the last bin."""
    h = np.asarray(h)
    out = 0.5 * h.copy()
    out[:-1] -= 0.25 * h[1:]
    out[1:] -= 0.25 * h[:-1]
    if h.size > 1:  # a one-bin grid: its missing neighbour is zero, as at the last bin
        out[0] -= 0.25 * np.conj(h[1])
    return out


def mismatch(a, b, S, w):
    """1 - sum_alpha <a|b>_alpha / sqrt(sum <a|a>_alpha sum <b|b>_alpha)
    over the two channels (the garbled Eq. mism read as a normalised
    overlap of the two-channel signal)."""
    from .likelihood import inner_product
    ab = sum(inner_product(x, y, S, w) for x, y in zip(a, b))
    aa = sum(inner_product(x, x, S, w) for x in a)
    bb = sum(inner_product(y, y, S, w) for y in b)
    return 1.0 - ab / np.sqrt(aa * bb)

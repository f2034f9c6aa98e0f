"""Downsampled frequency grids (oracle, test infrastructure).

Sec. 3.3: the FD waveform can be evaluated on an evenly spaced grid over
[0, f_max] only, f_max the largest frequency present in the signal, with
fewer bins than the DFT grid; the inner product then takes the grid's
spacing as its weight.  The band is the range of |F_V| over the ends of the
monotonic pieces of all voices; <h|h> on a grid is Eq. innerprod with that
weight, the DC bin excluded.
"""
from __future__ import annotations

import numpy as np

from .waveform import splines, voice_pieces, waveform


def signal_band(w):
    """(f_min, f_max): the smallest and largest |F_V| at piece ends."""
    sp = splines(w.traj, w.A)
    lo, hi = np.inf, 0.0
    for mi, ni in zip(w.m, w.n):
        cF = int(mi) * sp["Fphi"] + int(ni) * sp["Fr"]
        knotF = int(mi) * w.traj.Fphi + int(ni) * w.traj.Fr
        for _ta, _tb, Fa, Fb in voice_pieces(w.traj.t, cF, knotF):
            lo = min(lo, abs(Fa), abs(Fb))
            hi = max(hi, abs(Fa), abs(Fb))
    return (0.0 if lo == np.inf else lo), hi


def uniform_grid(f_max, n):
    """f_k = k f_max / n, k = 0..n."""
    return np.arange(n + 1) * (f_max / n)


def hh_on_grid(w, f, psd):
    """<h|h> summed over both channels on the grid f (spacing as weight)."""
    hp, hc = waveform(w, f=f)
    S = psd(f)
    df = f[1] - f[0]
    good = np.isfinite(S) & (f > 0)
    wS = np.zeros(f.size)
    wS[good] = 4.0 * df / S[good]
    return float(np.sum(wS * (np.abs(hp) ** 2 + np.abs(hc) ** 2)))

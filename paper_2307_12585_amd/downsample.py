"""Adaptive downsampled frequency grids (Sec. 3.3).

The FD waveform can be evaluated on an evenly spaced grid over [0, f_max]
only, f_max the largest frequency in the signal, with far fewer bins than the
DFT grid; the paper stresses that such a grid must be checked before it is
used.  adaptive_grid automates the check: it takes f_max from the device
(fdemri_signal_band), then doubles the bin count from n0 until <h|h> (the
fused likelihood with zero data, fdemri_loglike, so that no waveform is
stored) changes by at most tol between n and 2n bins, and returns the
n-bin grid with the sequence of <h|h> values it saw.
"""
from __future__ import annotations

import numpy as np
import torch

from . import DeviceWaveform


def uniform_grid(f_max, n):
    """f_k = k f_max / n, k = 0..n."""
    return np.arange(n + 1) * (f_max / n)


def hh_on_grid(ctx, w, f, psd, prec="fp64"):
    """<h|h> over both channels on grid f (spacing as the weight, DC excluded)."""
    dev = ctx.device
    dw = DeviceWaveform.from_workload(w, device=dev, f=f)
    S = psd(f)
    good = np.isfinite(S) & (f > 0)
    wS = np.zeros(f.size)
    wS[good] = 4.0 * (f[1] - f[0]) / S[good]
    ctype = torch.complex128 if prec == "fp64" else torch.complex64
    zero = torch.zeros(f.size, dtype=ctype, device=dev)
    out = ctx.loglike_dev(dw, zero, zero, torch.as_tensor(wS, device=dev), prec=prec)
    return float(out[1].cpu())


def adaptive_grid(ctx, w, psd, tol=1e-3, n0=64, n_max=1 << 22, prec="fp64"):
    """Smallest n = n0 2^j with |<h|h>_2n - <h|h>_n| <= tol <h|h>_2n on the
    uniform grid over [0, f_max]; returns (grid, [(n, <h|h>_n), ...])."""
    _, f_max = ctx.signal_band(DeviceWaveform.from_workload(w, device=ctx.device, f=np.array([0.0, 1.0])))
    n = n0
    hist = [(n, hh_on_grid(ctx, w, uniform_grid(f_max, n), psd, prec))]
    while n < n_max:
        hist.append((2 * n, hh_on_grid(ctx, w, uniform_grid(f_max, 2 * n), psd, prec)))
        if abs(hist[-1][1] - hist[-2][1]) <= tol * hist[-1][1]:
            return uniform_grid(f_max, n), hist
        n *= 2
    return uniform_grid(f_max, n), hist

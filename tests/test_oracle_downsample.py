"""Pins of the oracle's signal band and downsampled inner product: the band
of a linear chirp is its swept range exactly; on the DFT grid the
downsampled <h|h> is the inner product of Eq. innerprod; and for the
linear chirp <h|h> on any grid fine enough to resolve the band equals the
closed form 4 H^2 |c|^2 |fdot|^-1 int df / S over the band."""
import numpy as np

import workloads as W
from oracle.downsample import hh_on_grid, signal_band, uniform_grid
from oracle.likelihood import grid_weights, inner_product
from oracle.waveform import waveform


def test_band_of_linear_chirp():
    w = W.linear_chirp_workload()
    lo, hi = signal_band(w)
    f0, fdot, T = 2e-3, 1e-10, 2e6
    assert abs(lo - f0) <= 1e-15 * f0 and abs(hi - (f0 + fdot * T)) <= 1e-14 * hi


def test_hh_on_dft_grid_is_the_inner_product():
    w = W.inspiral_20_modes()
    f = w.f[:20001]
    S = W.psd_closed_form(f)
    hp, hc = waveform(w, f=f)
    ref = inner_product(hp, hp, S, grid_weights(f)) + inner_product(hc, hc, S, grid_weights(f))
    assert abs(hh_on_grid(w, f, W.psd_closed_form) - ref) <= 1e-12 * ref


def test_hh_of_linear_chirp_closed_form():
    # |h~_+(f)|^2 = |A c_+|^2 / |fdot| inside the band for one voice (the
    # Fresnel transform), so <h|h> = 4 (|A c_+|^2 + |A c_x|^2) / |fdot| int df/S
    w = W.linear_chirp_workload()
    f0, fdot, T = 2e-3, 1e-10, 2e6
    S0 = 2.0e-40
    psd = lambda f: np.full(f.size, S0)
    f = uniform_grid(signal_band(w)[1] * 1.0001, 40000)
    hh = hh_on_grid(w, f, psd)
    hp, hc = waveform(w, f=np.array([f0 + 0.5 * fdot * T]))
    # |h~|^2 at an interior bin times the band width
    ref = 4.0 * (abs(hp[0]) ** 2 + abs(hc[0]) ** 2) * (fdot * T) / S0
    assert abs(hh - ref) <= 2e-3 * ref

"""The signal band (fdemri_signal_band) and the adaptive downsampled grid
(paper_2307_12585_amd.downsample) against the oracle's band and its <h|h>
on the same grids."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.downsample import hh_on_grid as oracle_hh
from oracle.downsample import signal_band as oracle_band

pytestmark = pytest.mark.gpu
fd = pytest.importorskip("paper_2307_12585_amd")


@pytest.fixture(scope="module")
def ctx():
    c = fd.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name", ["inspiral_20_modes", "inspiral_3842_modes", "linear_chirp_workload"])
def test_signal_band_matches_oracle(ctx, name):
    w = getattr(W, name)()
    lo, hi = ctx.signal_band(fd.DeviceWaveform.from_workload(w, device=ctx.device))
    rlo, rhi = oracle_band(w)
    print(name, (lo, hi), (rlo, rhi))
    assert abs(hi - rhi) <= 1e-13 * rhi
    assert abs(lo - rlo) <= 1e-13 * max(rlo, 1e-300) or (rlo == 0 and lo == 0)


def test_adaptive_grid_20_modes(ctx):
    from paper_2307_12585_amd.downsample import adaptive_grid, uniform_grid
    w = W.inspiral_20_modes()
    grid, hist = adaptive_grid(ctx, w, W.psd_closed_form, tol=1e-3, n0=64)
    print("chosen bins", grid.size - 1, "history", hist)
    f_max = oracle_band(w)[1]
    for n, hh in hist:
        ref = oracle_hh(w, uniform_grid(f_max, n), W.psd_closed_form)
        assert abs(hh - ref) <= 1e-9 * ref, (n, hh, ref)
    (n1, h1), (n2, h2) = hist[-2], hist[-1]
    assert n1 == grid.size - 1 and abs(h2 - h1) <= 1e-3 * h2
    # against the full DFT grid
    full = oracle_hh(w, w.f, W.psd_closed_form)
    print("downsampled <h|h>", h1, "full grid", full, "bins", grid.size - 1, "of", w.f.size)

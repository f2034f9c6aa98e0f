"""fdemri_td_waveform (through the C ABI): the time-domain voice sum against
the oracle's time-domain sum, and its Hann-windowed transform against the
frequency-domain sum (the paper's FD/TD comparison; the mismatch of Eq. mism,
read as R12)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.likelihood import grid_weights
from oracle.td import fd_hann, hann, mismatch, td_waveform
from oracle.waveform import splines

pytestmark = pytest.mark.gpu
fd = pytest.importorskip("paper_2307_12585_amd")
from gpu_helpers import gpu_waveform, rel_l2  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = fd.Context(0)
    yield c
    c.close()


def gpu_td(ctx, w, t0, dt, Nt):
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    hp, hc = ctx.td_waveform_dev(dw, t0, dt, Nt)
    torch.cuda.synchronize()
    return hp.cpu().numpy(), hc.cpu().numpy()


def phase_bound(w):
    """Largest |m Phi_phi + n Phi_r| over the trajectory: the oracle forms it
    in plain FP64, so its phase error is a few units of this times 2^-52."""
    return float(np.max(np.abs(w.m[:, None] * w.traj.Phiphi[None, :] + w.n[:, None] * w.traj.Phir[None, :])))


def test_td_matches_oracle_20_modes(ctx):
    w = W.inspiral_20_modes()
    dt = w.meta["dt"]
    Nt = int(round(w.meta["T"] / dt))
    hp, hc = gpu_td(ctx, w, 0.0, dt, Nt)
    h = td_waveform(w, np.arange(Nt) * dt)
    tol = 20 * phase_bound(w) * 2.0 ** -52
    e = (rel_l2(hp, h.real), rel_l2(hc, -h.imag))
    print("TD rel L2", e, "tol", tol)
    assert max(e) <= tol


def test_td_grid_edges_and_no_partners(ctx):
    w = W.inspiral_20_modes()
    tend = w.traj.t[-1]
    dt = 977.0
    t0 = -5 * dt - 1.5
    Nt = int((tend - t0) / dt) + 7   # samples before, inside and after the trajectory
    hp, hc = gpu_td(ctx, w, t0, dt, Nt)
    ts = t0 + np.arange(Nt) * dt
    h = td_waveform(w, ts)
    out = (ts < 0) | (ts > tend)
    assert np.all(hp[out] == 0) and np.all(hc[out] == 0)
    tol = 20 * phase_bound(w) * 2.0 ** -52
    assert rel_l2(hp, h.real) <= tol and rel_l2(hc, -h.imag) <= tol
    # single voices of either sign of m
    w2 = W.inspiral_20_modes()
    sel = np.arange(6)
    w2.l, w2.n, w2.A = w2.l[sel], w2.n[sel], w2.A[sel]
    w2.m = np.array([2, -2, 2, -2, 2, -2], np.int32)
    dw = fd.DeviceWaveform.from_workload(w2, device=ctx.device, partners=False)
    gp, gc = ctx.td_waveform_dev(dw, 0.0, dt, Nt // 2)
    torch.cuda.synchronize()
    h2 = td_waveform(w2, np.arange(Nt // 2) * dt, partners=False)
    assert rel_l2(gp.cpu().numpy(), h2.real) <= tol and rel_l2(gc.cpu().numpy(), -h2.imag) <= tol
    # no samples
    e = torch.zeros(1, dtype=torch.float64, device=ctx.device)
    ctx.td_waveform_dev(fd.DeviceWaveform.from_workload(w, device=ctx.device), 0.0, dt, 0, out=(e[:0], e[:0]))


@pytest.mark.parametrize("name", ["inspiral_20_modes", "inspiral_3842_modes"])
def test_td_transform_against_fd_sum(ctx, name):
    """The Hann-windowed transform of the TD sum against the FD sum convolved
    with the matching three-tap kernel (R11, R18): the mismatch measures the
    stationary-phase approximation itself."""
    w = getattr(W, name)()
    dt = w.meta["dt"]
    Nt = 2 * (w.f.size - 1)
    hp, hc = gpu_td(ctx, w, 0.0, dt, Nt)
    win = hann(Nt)
    tp = dt * np.conj(np.fft.rfft(hp * win))
    tc = dt * np.conj(np.fft.rfft(hc * win))
    fp, fc = gpu_waveform(ctx, w)
    S = W.psd_closed_form(w.f)
    mm = mismatch((fd_hann(fp), fd_hann(fc)), (tp, tc), S, grid_weights(w.f))
    print(name, "FD/TD mismatch", mm)
    assert mm <= 5e-3

"""The fused Whittle log-likelihood (fdemri_loglike, through the C ABI)
against the oracle's sums: on the oracle's own waveform (the FP64 bar carried
through a Cauchy-Schwarz bound) and on the GPU's stored waveform (then the
fusion alone is under test, to summation order), with and without the
frequency-domain Hann kernel, in FP64 and mixed precision."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle.likelihood import fused_sums, grid_weights
from oracle.td import fd_hann

pytestmark = pytest.mark.gpu
fd = pytest.importorskip("paper_2307_12585_amd")
from gpu_helpers import gpu_waveform  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = fd.Context(0)
    yield c
    c.close()


def weights(f):
    S = W.psd_closed_form(f)
    w = grid_weights(f)
    good = np.isfinite(S) & (w > 0)
    return np.where(good, 4.0 * w / np.where(good, S, 1.0), 0.0)


def data_for(h, f, seed):
    """Scaled, phase-shifted model plus noise of the closed-form PSD."""
    df = float(f[1] - f[0]) if f.size > 1 else 1.0
    n_p, n_c = W.noise_draw(f, df, seed)
    return (1.1 * np.exp(0.3j) * h[0] + n_p, 0.9 * np.exp(-0.2j) * h[1] + n_c)


def gpu_loglike(ctx, w, d, wS, prec="fp64", hann=False, f=None, flags=0):
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device, f=f)
    ctype = torch.complex128 if prec == "fp64" else torch.complex64
    dp = torch.as_tensor(d[0], device=ctx.device).to(ctype).contiguous()
    dc = torch.as_tensor(d[1], device=ctx.device).to(ctype).contiguous()
    ws = torch.as_tensor(wS, dtype=torch.float64, device=ctx.device).contiguous()
    out = ctx.loglike_dev(dw, dp, dc, ws, prec=prec, hann=hann)
    torch.cuda.synchronize()
    assert ctx.sync_flags() == flags
    return out.cpu().numpy()


def close(a, b, tol):
    return abs(a - b) <= tol * max(abs(b), 1e-300)


@pytest.mark.parametrize("hann", [False, True])
def test_loglike_matches_oracle_20_modes(ctx, hann):
    w = W.inspiral_20_modes()
    ho = oracle.waveform(w)
    wS = weights(w.f)
    d = data_for(ho, w.f, 7)
    ref = fused_sums(d, ho, wS, hann=hann)
    got = gpu_loglike(ctx, w, d, wS, hann=hann)
    # against the oracle's model: the model error enters log L through
    # |d - h| |dh| (Cauchy-Schwarz) and <h|h>, <d|h> through |h| |dh|, |d| |dh|
    hg = gpu_waveform(ctx, w)
    g = [fd_hann(x) if hann else x for x in hg]
    o = [fd_hann(x) if hann else x for x in ho]
    dh = np.sqrt(sum(np.sum(wS * np.abs(a - b) ** 2) for a, b in zip(g, o)))
    nh = np.sqrt(sum(np.sum(wS * np.abs(b) ** 2) for b in o))
    nd = np.sqrt(sum(np.sum(wS * np.abs(x) ** 2) for x in d))
    print("gpu", got, "oracle", ref, "model error", dh / nh)
    assert abs(got[0] - ref[0]) <= 1.01 * np.sqrt(-2 * ref[0]) * dh + 1e-12 * abs(ref[0])
    assert abs(got[1] - ref[1]) <= 1.01 * (2 * nh + dh) * dh + 1e-12 * ref[1]
    assert abs(got[2] - ref[2]) <= 1.01 * nd * dh + 1e-12 * abs(ref[2])
    # against the oracle's sums of the GPU's stored waveform: the fusion alone
    ref_g = fused_sums(d, hg, wS, hann=hann)
    for q in range(3):
        assert close(got[q], ref_g[q], 1e-12), (q, got[q], ref_g[q])


@pytest.mark.parametrize("hann", [False, True])
def test_loglike_mixed_against_stored_mixed_waveform(ctx, hann):
    w = W.inspiral_20_modes()
    hm = gpu_waveform(ctx, w, prec="mixed")
    wS = weights(w.f)
    d = data_for(oracle.waveform(w), w.f, 8)
    d32 = tuple(x.astype(np.complex64).astype(np.complex128) for x in d)
    got = gpu_loglike(ctx, w, d, wS, prec="mixed", hann=hann)
    ref = fused_sums(d32, [x.astype(np.complex128) for x in hm], wS, hann=hann)
    for q in range(3):
        assert close(got[q], ref[q], 1e-12), (q, got[q], ref[q])
    # and within the mixed bar of the FP64 fused result
    got64 = gpu_loglike(ctx, w, d, wS, hann=hann)
    assert close(got[0], got64[0], 1e-6) and close(got[1], got64[1], 1e-6)


@pytest.mark.parametrize("hann", [False, True])
def test_loglike_3842_modes_fused_equals_unfused(ctx, hann):
    """Full size: the fused sums equal the oracle's sums of the stored GPU
    waveform (every tile's edge records, blocks outside the envelope)."""
    w = W.inspiral_3842_modes()
    hg = gpu_waveform(ctx, w)
    wS = weights(w.f)
    d = data_for(hg, w.f, 9)
    got = gpu_loglike(ctx, w, d, wS, hann=hann)
    ref = fused_sums(d, hg, wS, hann=hann)
    print("gpu", got, "ref", ref)
    for q in range(3):
        assert close(got[q], ref[q], 1e-11), (q, got[q], ref[q])


def test_loglike_ragged_and_offset_grids(ctx):
    """Ragged grid lengths (the Hann edge records across tiles and at the grid
    end) on DFT grids from f = 0, with and without the Hann kernel; offset
    grids without it.  The Hann kernel on an offset grid (not f_k = k f_1)
    raises FDEMRI_FLAG_BAD_INPUT and compares the data with a zero model."""
    w = W.inspiral_20_modes()
    rng = np.random.default_rng(3)
    grids = [(0, 1), (0, 63), (0, 64), (0, 65), (0, 257), (0, 1000), (0, 65 * 64 + 3), (0, 100001 + 65 * 64 + 3),
             (3, 1000), (12345, 12345 + 257), (100001, 100001 + 65 * 64 + 3)]
    for lo, hi in grids:
        f = w.f[lo:hi]
        hg = gpu_waveform(ctx, w, f=f)
        wS = rng.uniform(0.5, 2.0, f.size)
        d = tuple(rng.normal(size=f.size) + 1j * rng.normal(size=f.size) for _ in range(2))
        scale = max(np.max(np.abs(hg[0])), 1e-30)
        d = tuple(x * scale for x in d)
        for hann in (False, True):
            dft = lo == 0
            if hann and not dft:
                got = gpu_loglike(ctx, w, d, wS, hann=True, f=f, flags=fd.FDEMRI_FLAG_BAD_INPUT)
                zero = tuple(np.zeros(f.size, complex) for _ in range(2))
                ref = fused_sums(d, zero, wS, hann=True)
                assert got[1] == 0.0 and got[2] == 0.0
                assert abs(got[0] - ref[0]) <= 1e-12 * abs(ref[0]), (lo, hi)
                continue
            got = gpu_loglike(ctx, w, d, wS, hann=hann, f=f)
            ref = fused_sums(d, hg, wS, hann=hann)
            for q in range(3):
                tol = 1e-12 * max(abs(ref[q]), abs(ref[0]), abs(ref[1]))
                assert abs(got[q] - ref[q]) <= tol, (lo, hi, hann, q, got[q], ref[q])


def test_loglike_deterministic_and_invalid(ctx):
    w = W.inspiral_20_modes()
    wS = weights(w.f)
    d = data_for(oracle.waveform(w), w.f, 1)
    a = gpu_loglike(ctx, w, d, wS, hann=True)
    b = gpu_loglike(ctx, w, d, wS, hann=True)
    assert np.array_equal(a, b)
    # NULL data or output, unknown flags: EINVAL, nothing enqueued
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    desc = dw.desc()
    import ctypes
    lib = fd.lib()
    out = torch.zeros(3, dtype=torch.float64, device=ctx.device)
    st = lib.fdemri_loglike(ctx._h, ctypes.byref(desc), 0, None, None, None, 0, out.data_ptr(), None)
    assert st == 1
    ws = torch.as_tensor(wS, device=ctx.device)
    dp = torch.zeros(w.Nf, dtype=torch.complex128, device=ctx.device)
    st = lib.fdemri_loglike(ctx._h, ctypes.byref(desc), 0, dp.data_ptr(), dp.data_ptr(), ws.data_ptr(), 0x10,
                            out.data_ptr(), None)
    assert st == 1
    torch.cuda.synchronize()
    assert torch.all(out == 0)


@pytest.mark.parametrize("prec,hann", [("fp64", False), ("fp64", True), ("mixed", True)])
def test_loglike_batch_equals_single_calls(ctx, prec, hann):
    """fdemri_loglike_batch over waveforms of uneven sizes (ragged grids, a
    log grid) equals one fdemri_loglike call per waveform, bit for bit.""" 
    ws = [W.inspiral_20_modes(), W.inspiral_20_modes_log_grid()]
    for prm in W.batch_params(3, 321):
        prm["T"] = min(prm["T"], 0.6 * W.YRSID_SI)
        w = W.batch_workload(prm, K=70 + 10 * len(ws))
        w.f = w.f[: 120_000 + 37 * len(ws)]
        ws.append(w)
    ctype = torch.complex128 if prec == "fp64" else torch.complex64
    rng = np.random.default_rng(17)
    dws, dps, dcs, wss = [], [], [], []
    for w in ws:
        dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
        hp, hc = ctx.waveform_dev(dw, "fp64")
        noise = [torch.as_tensor(rng.normal(size=(w.Nf, 2)), device=ctx.device) for _ in range(2)]
        sc = float(torch.max(torch.abs(hp))) + 1e-30
        dps.append((1.2 * hp + sc * torch.view_as_complex(noise[0])).to(ctype).contiguous())
        dcs.append((0.8 * hc + sc * torch.view_as_complex(noise[1])).to(ctype).contiguous())
        wss.append(torch.as_tensor(rng.uniform(0.5, 2.0, w.Nf), device=ctx.device))
        dws.append(dw)
    out = ctx.loglike_batch(dws, dps, dcs, wss, prec=prec, hann=hann)
    torch.cuda.synchronize()
    # the log-grid member is not a DFT grid: with the Hann kernel it is flagged
    # and compared with a zero model, in the batch as in its single call
    assert ctx.sync_flags() == (fd.FDEMRI_FLAG_BAD_INPUT if hann else 0)
    if hann:
        assert float(out[1, 1]) == 0.0 and float(out[1, 2]) == 0.0 and float(out[0, 1]) > 0
    for b, dw in enumerate(dws):
        single = ctx.loglike_dev(dw, dps[b], dcs[b], wss[b], prec=prec, hann=hann)
        torch.cuda.synchronize()
        assert torch.equal(out[b], single), (b, out[b], single)

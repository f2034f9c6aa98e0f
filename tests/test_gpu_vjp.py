"""The HIP adjoint (fdemri_vjp, through the C ABI) against the oracle's
gradient and against central finite differences of the HIP forward."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.gradient import coef_grad_to_knots, waveform_vjp

pytestmark = pytest.mark.gpu
fd = pytest.importorskip("paper_2307_12585_amd")
from gpu_helpers import rel_l2  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = fd.Context(0)
    yield c
    c.close()


def small_workload(stride=9):
    w = W.inspiral_20_modes()
    sel = np.array([2, 6, 9, 13])
    w.l, w.m, w.n, w.A = w.l[sel], w.m[sel], w.n[sel], w.A[sel]
    w.f = w.f[::stride]
    return w


def cotangents(n, seed):
    rng = np.random.default_rng(seed)
    return [(rng.normal(size=n) + 1j * rng.normal(size=n)) * 1e20 for _ in range(2)]


@pytest.mark.parametrize("partners", [True, False])
def test_vjp_matches_oracle(ctx, partners):
    w = small_workload()
    if not partners:
        w.m = np.array([2, -2, 2, -2], np.int32)
    g_p, g_c = cotangents(w.Nf, 3)
    ref = waveform_vjp(w, g_p, g_c, partners=partners)
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device, partners=partners)
    out = ctx.vjp_dev(dw, torch.as_tensor(g_p, device=ctx.device), torch.as_tensor(g_c, device=ctx.device))
    torch.cuda.synchronize()
    gA = out["gA"].cpu().numpy()
    gPhi = out["gPhi"].cpu().numpy()
    gsc = out["g_scalars"].cpu().numpy()
    print("gA", rel_l2(gA, ref["gA"]), "gPhi", rel_l2(gPhi[0], ref["gPhi"][0]), rel_l2(gPhi[1], ref["gPhi"][1]))
    print("scalars", gsc, ref["g_scalars"])
    assert rel_l2(gA, ref["gA"]) <= 1e-9
    for r in range(2):
        for k in range(4):
            assert rel_l2(gPhi[r, :, k], ref["gPhi"][r, :, k]) <= 1e-8
    for q in range(5):
        assert abs(gsc[q] - ref["g_scalars"][q]) <= 1e-9 * max(abs(ref["g_scalars"][q]), 1e-300)
    kn = coef_grad_to_knots(w.traj.t, ref["gA"])
    assert rel_l2(out["gA_knots"].cpu().numpy(), kn) <= 1e-9
    knp = coef_grad_to_knots(w.traj.t, ref["gPhi"])
    assert rel_l2(out["gPhi_knots"].cpu().numpy(), knp) <= 1e-8


def test_vjp_matches_oracle_at_max_knots(ctx):
    """The adjoint and its transposed spline solve at FDEMRI_MAX_KNOTS knots."""
    w0 = W.inspiral_20_modes(K=512)
    sel = np.array([2, 9])
    w0.l, w0.m, w0.n, w0.A = w0.l[sel], w0.m[sel], w0.n[sel], w0.A[sel]
    w0.f = w0.f[::5]
    g_p, g_c = cotangents(w0.Nf, 4)
    ref = waveform_vjp(w0, g_p, g_c)
    dw = fd.DeviceWaveform.from_workload(w0, device=ctx.device)
    out = ctx.vjp_dev(dw, torch.as_tensor(g_p, device=ctx.device), torch.as_tensor(g_c, device=ctx.device))
    torch.cuda.synchronize()
    assert rel_l2(out["gA"].cpu().numpy(), ref["gA"]) <= 1e-9
    kn = coef_grad_to_knots(w0.traj.t, ref["gA"])
    assert rel_l2(out["gA_knots"].cpu().numpy(), kn) <= 1e-9
    knp = coef_grad_to_knots(w0.traj.t, ref["gPhi"])
    assert rel_l2(out["gPhi_knots"].cpu().numpy(), knp) <= 1e-8


def _whittle(hp, hc, dp, dc, S, wts):
    L = 0.0
    for h, d in ((hp, dp), (hc, dc)):
        L = L - 0.5 * 4.0 * torch.sum(wts * torch.abs(d - h) ** 2 / S)
    return L


def test_vjp_central_differences_of_gpu_forward(ctx):
    """Directional derivative of the Whittle loss through the HIP forward (FP64)
    against the HIP gradient (knot values, angles, scale), rel <= 1e-5."""
    w = small_workload(stride=3)
    dev = ctx.device
    f = torch.as_tensor(w.f, device=dev)
    S = torch.as_tensor(np.where(np.isfinite(W.psd_closed_form(w.f)), W.psd_closed_form(w.f), np.inf), device=dev)
    wts = torch.full_like(f, float(w.f[1] - w.f[0]))
    wts[0] = 0
    dw = fd.DeviceWaveform.from_workload(w, device=dev)
    hp, hc = ctx.waveform_dev(dw)
    dp, dc = 1.05 * hp.clone(), 0.97 * hc.clone()
    g_p = 4 * wts * (dp - hp) / S
    g_c = 4 * wts * (dc - hc) / S
    out = ctx.vjp_dev(dw, g_p, g_c)
    rng = np.random.default_rng(0)
    dA = torch.as_tensor((rng.normal(size=w.A.shape) + 1j * rng.normal(size=w.A.shape)) * np.abs(w.A), device=dev)
    dP = torch.as_tensor(rng.normal(size=(2, w.K)) * 1e-3, device=dev)
    dth, dph, dsc = 0.3, -0.2, 0.1 * w.scale

    def loss(e):
        d2 = fd.DeviceWaveform.from_workload(w, device=dev)
        d2.A = torch.view_as_real(torch.view_as_complex(dw.A) + e * dA).contiguous()
        d2.Phiphi = dw.Phiphi + e * dP[0]
        d2.Phir = dw.Phir + e * dP[1]
        d2.theta, d2.phi, d2.scale = w.theta + e * dth, w.phi + e * dph, w.scale + e * dsc
        h2p, h2c = ctx.waveform_dev(d2)
        return float(_whittle(h2p, h2c, dp, dc, S, wts))
    eps = 1e-4
    num = (loss(eps) - loss(-eps)) / (2 * eps)
    ana = float(torch.sum((torch.conj(out["gA_knots"]) * dA).real)
                + torch.sum(out["gPhi_knots"] * dP)
                + out["g_scalars"][0] * dth + out["g_scalars"][1] * dph + out["g_scalars"][2] * dsc)
    print("FD", num, "analytic", ana)
    assert abs(num - ana) <= 1e-5 * abs(ana)


def test_vjp_mixed_against_fp64(ctx):
    w = small_workload(stride=3)
    g_p, g_c = cotangents(w.Nf, 5)
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    gp = torch.as_tensor(g_p, device=ctx.device)
    gc = torch.as_tensor(g_c, device=ctx.device)
    a = ctx.vjp_dev(dw, gp, gc, "fp64")
    b = ctx.vjp_dev(dw, gp.to(torch.complex64), gc.to(torch.complex64), "mixed")
    for key in ("gA", "gPhi", "gA_knots", "g_scalars"):
        err = rel_l2(b[key].cpu().numpy(), a[key].cpu().numpy())
        print("mixed vs fp64", key, err)
        assert err <= 1e-5


def test_vjp_deterministic(ctx):
    w = small_workload()
    g_p, g_c = cotangents(w.Nf, 7)
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    gp = torch.as_tensor(g_p, device=ctx.device)
    gc = torch.as_tensor(g_c, device=ctx.device)
    a = ctx.vjp_dev(dw, gp, gc)
    b = ctx.vjp_dev(dw, gp, gc)
    for key in a:
        assert torch.equal(a[key], b[key])


def test_autograd_gradcheck(ctx):
    """torch.autograd.gradcheck of the waveform through FDEmriFn (FP64) on a
    tiny input: 12 knots, 2 modes, ~60 bins."""
    from paper_2307_12585_amd.autograd import WaveformStatic, fdemri_waveform
    w = W.inspiral_20_modes(K=12)
    w.l, w.m, w.n, w.A = w.l[[6, 9]], w.m[[6, 9]], w.n[[6, 9]], w.A[[6, 9]]
    sel = np.nonzero((w.f > 0) & (np.arange(w.Nf) % 97 == 0))[0]
    dev = ctx.device
    st = WaveformStatic(w.traj.t, w.traj.Fphi, w.traj.Fr, w.l, w.m, w.n, w.f[sel], device=dev)
    A = torch.as_tensor(w.A, device=dev).requires_grad_(True)
    Pp = torch.as_tensor(w.traj.Phiphi, device=dev).requires_grad_(True)
    Pr = torch.as_tensor(w.traj.Phir, device=dev).requires_grad_(True)
    th = torch.tensor(w.theta, dtype=torch.float64, device=dev, requires_grad=True)
    ph = torch.tensor(w.phi, dtype=torch.float64, device=dev, requires_grad=True)
    sc = torch.tensor(1.0, dtype=torch.float64, device=dev, requires_grad=True)

    def fn(A, Pp, Pr, th, ph, sc):
        hp, hc = fdemri_waveform(ctx, st, A, Pp, Pr, th, ph, sc)
        return hp * 1e-6, hc * 1e-6
    assert torch.autograd.gradcheck(fn, (A, Pp, Pr, th, ph, sc), eps=1e-6, atol=1e-7, rtol=1e-4)


def test_autograd_whittle_backward(ctx):
    """loss.backward() through FDEmriFn equals the library VJP on the Whittle
    cotangent."""
    from paper_2307_12585_amd.autograd import WaveformStatic, fdemri_waveform, whittle_loglike
    w = small_workload(stride=5)
    dev = ctx.device
    st = WaveformStatic(w.traj.t, w.traj.Fphi, w.traj.Fr, w.l, w.m, w.n, w.f, device=dev)
    A = torch.as_tensor(w.A, device=dev).requires_grad_(True)
    Pp = torch.as_tensor(w.traj.Phiphi, device=dev).requires_grad_(True)
    Pr = torch.as_tensor(w.traj.Phir, device=dev).requires_grad_(True)
    th = torch.tensor(w.theta, dtype=torch.float64, device=dev, requires_grad=True)
    hp, hc = fdemri_waveform(ctx, st, A, Pp, Pr, th, w.phi, w.scale)
    S = torch.as_tensor(W.psd_closed_form(w.f), device=dev)
    wts = torch.full_like(S, float(w.f[1] - w.f[0]))
    wts[0] = 0
    # data with a phase offset, so that the phase gradients do not cancel
    dp = (1.1 * hp * np.exp(0.3j)).detach()
    dc = (0.9 * hc * np.exp(-0.2j)).detach()
    L = whittle_loglike(hp, hc, dp, dc, S, wts)
    L.backward()
    g_p = (4 * wts * (dp - hp) / S).detach()
    g_c = (4 * wts * (dc - hc) / S).detach()
    dw = fd.DeviceWaveform.from_workload(w, device=dev)
    ref = ctx.vjp_dev(dw, g_p, g_c)
    # the two cotangents differ by rounding of the loss derivative; the phase
    # gradients sum terms of both signs, so compare in relative L2
    rl = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    assert rl(A.grad, ref["gA_knots"]) <= 1e-12
    assert rl(Pp.grad, ref["gPhi_knots"][0]) <= 1e-9
    assert abs(float(th.grad) - float(ref["g_scalars"][0])) <= 1e-9 * abs(float(ref["g_scalars"][0]))


def _compare_with_oracle(out, ref, t, what, tol_a=1e-9, tol_p=1e-8):
    """The HIP gradient groups against the oracle's (coefficients, knots,
    scalars); each scalar to tol_a relative, or to tol_a of the largest
    scalar of its kind where the oracle's value is zero."""
    gA = out["gA"].cpu().numpy()
    gPhi = out["gPhi"].cpu().numpy()
    gsc = out["g_scalars"].cpu().numpy()
    print(what, "gA", rel_l2(gA, ref["gA"]), "gPhi", rel_l2(gPhi, ref["gPhi"]), "scalars", gsc, ref["g_scalars"])
    assert np.linalg.norm(ref["gA"]) > 0
    assert rel_l2(gA, ref["gA"]) <= tol_a, what
    for r in range(2):
        for k in range(4):
            assert rel_l2(gPhi[r, :, k], ref["gPhi"][r, :, k]) <= tol_p, (what, r, k)
    for q in range(5):
        scale = abs(ref["g_scalars"][q]) if ref["g_scalars"][q] != 0 else np.max(np.abs(ref["g_scalars"]))
        assert abs(gsc[q] - ref["g_scalars"][q]) <= tol_a * scale, (what, q)
    assert rel_l2(out["gA_knots"].cpu().numpy(), coef_grad_to_knots(t, ref["gA"])) <= tol_a, what
    assert rel_l2(out["gPhi_knots"].cpu().numpy(), coef_grad_to_knots(t, ref["gPhi"])) <= tol_p, what


def _turnover_and_crossing_voices():
    from test_oracle_waveform import turnover_workload, zero_crossing_workload
    return {
        "turnover on a knot": turnover_workload(1e-2, 1e-9),
        "turnover inside a segment": turnover_workload(6e-2, -1e-9, K=40),
        "zero crossing between knots": zero_crossing_workload(1e-9, False)[0],
        "zero crossing on a knot": zero_crossing_workload(-1e-9, True)[0],
    }


@pytest.mark.parametrize("partners", [False, True])
@pytest.mark.parametrize("name", ["turnover on a knot", "turnover inside a segment",
                                  "zero crossing between knots", "zero crossing on a knot"])
def test_vjp_matches_oracle_turnover_and_zero_crossing(ctx, name, partners):
    """The adjoint where a bin has two roots (a turnover: both monotonic
    pieces of the voice own the bin, in the same or in adjacent segments) and
    where the voice frequency crosses zero (the F_V < 0 piece feeds h(-f),
    with the conjugated amplitude and the opposite phase sign): against the
    oracle's term-by-term gradient, with and without the partner voice."""
    w = _turnover_and_crossing_voices()[name]
    g_p, g_c = cotangents(w.Nf, 11)
    g_p, g_c = g_p * 1e-20, g_c * 1e-20
    ref = waveform_vjp(w, g_p, g_c, partners=partners)
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device, partners=partners)
    out = ctx.vjp_dev(dw, torch.as_tensor(g_p, device=ctx.device), torch.as_tensor(g_c, device=ctx.device))
    torch.cuda.synchronize()
    assert ctx.sync_flags() == 0
    _compare_with_oracle(out, ref, w.traj.t, f"{name}, partners={partners}")


def _cfg5_draw(k):
    """Draw k of the forward+adjoint workload (the batch distribution, seed 1)."""
    return W.batch_workload(W.batch_params(64, 1)[k])


def test_vjp_dense_draw_sampled_cotangent(ctx):
    """A draw of the forward+adjoint workload with the densest bins among its
    first eight (the smallest M), one mode row in 13, on its whole grid, with
    a cotangent that is zero except on 2000 sampled bins: the HIP adjoint
    against the oracle's gradient evaluated on those bins only (bins with a
    zero cotangent contribute nothing).  Here the root solve continues past
    its first Halley step and the segment walks run on most lanes."""
    prms = W.batch_params(64, 1)[:8]
    k = int(np.argmin([p["M"] for p in prms]))
    w = _cfg5_draw(k)
    sel = np.arange(0, w.Nm, 13)
    w.l, w.m, w.n, w.A = w.l[sel], w.m[sel], w.n[sel], w.A[sel]
    rng = np.random.default_rng(21)
    idx = np.sort(rng.choice(np.arange(1, w.Nf), 2000, replace=False))
    gs_p, gs_c = cotangents(idx.size, 22)
    ref = waveform_vjp(w, gs_p, gs_c, f=w.f[idx])
    g_p = np.zeros(w.Nf, np.complex128)
    g_c = np.zeros(w.Nf, np.complex128)
    g_p[idx], g_c[idx] = gs_p, gs_c
    dw = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    out = ctx.vjp_dev(dw, torch.as_tensor(g_p, device=ctx.device), torch.as_tensor(g_c, device=ctx.device))
    torch.cuda.synchronize()
    assert ctx.sync_flags() == 0
    _compare_with_oracle(out, ref, w.traj.t, f"draw {k} (M = {prms[k]['M']:.3g}), {w.Nm} rows, 2000 bins")


@pytest.mark.parametrize("k", [0, 1, 2, 3, 10, 14])
def test_vjp_central_differences_on_forward_adjoint_draws(ctx, k):
    """The first four draws of the forward+adjoint workload, and draws 10
    (M = 1.1e5: 1.8e9 group-bin evaluations, so chunks longer than the
    minimum) and 14 (single (group, segment) units of hundreds of thousands
    of bins, split into hundreds of chunks), at full size (all
    kept modes, whole grid): the Whittle log-likelihood of data = waveform at
    the draw + noise of the closed-form PSD, for a template with perturbed
    amplitudes, Phi_phi offset and inclination; each gradient group (amplitude
    knots, phase knots, theta, phi, scale, Phi_phi0, Phi_r0) against the
    central difference of the HIP FP64 forward along a seeded direction,
    rel <= 1e-5."""
    import dataclasses
    w = _cfg5_draw(k)
    dev = ctx.device
    df = float(w.f[1] - w.f[0])
    S = W.psd_closed_form(w.f)
    wS = torch.as_tensor(np.where(np.isfinite(S), 4.0 * df / np.where(np.isfinite(S), S, 1.0), 0.0), device=dev)
    hp0, hc0 = ctx.waveform_dev(fd.DeviceWaveform.from_workload(w, device=dev))
    n1, n2 = W.noise_draw(w.f, df, 100 + k)
    dp = hp0 + torch.as_tensor(n1, device=dev)
    dc = hc0 + torch.as_tensor(n2, device=dev)
    traj = dataclasses.replace(w.traj, Phiphi=w.traj.Phiphi + 0.3)
    tpl = dataclasses.replace(w, traj=traj, A=w.A * (1.02 * np.exp(0.05j)), theta=w.theta + 0.01)
    dw = fd.DeviceWaveform.from_workload(tpl, device=dev)

    def loss(d2):
        h2p, h2c = ctx.waveform_dev(d2)
        return -0.5 * float(torch.sum(wS * (torch.abs(dp - h2p) ** 2 + torch.abs(dc - h2c) ** 2)))

    hp, hc = ctx.waveform_dev(dw)
    out = ctx.vjp_dev(dw, wS * (dp - hp), wS * (dc - hc))
    torch.cuda.synchronize()
    assert ctx.sync_flags() == 0
    rng = np.random.default_rng(200 + k)
    dA = torch.as_tensor((rng.normal(size=tpl.A.shape) + 1j * rng.normal(size=tpl.A.shape)) * np.abs(tpl.A), device=dev)
    dP = torch.as_tensor(rng.normal(size=(2, w.K)), device=dev)
    gsc = out["g_scalars"].cpu().numpy()

    # The knot phases reach ~1e6 rad, where a step of 1e-5 rad is stored to
    # ~1e-10 rad only: the directional derivative is taken along the step
    # actually stored, fl(x + e v) - x (exact, by Sterbenz), on both sides.
    ones = torch.ones(w.K, dtype=torch.float64, device=dev)

    def shifted(e, group):
        """Perturbed inputs and the adjoint's prediction of the loss change."""
        d2 = fd.DeviceWaveform.from_workload(tpl, device=dev)
        if group == "amplitudes":
            d2.A = torch.view_as_real(torch.view_as_complex(dw.A) + e * dA).contiguous()
            pred = float(torch.sum((torch.conj(out["gA_knots"]) * (torch.view_as_complex(d2.A) - torch.view_as_complex(dw.A))).real))
        elif group in ("phases", "Phi_phi0", "Phi_r0"):
            v = {"phases": dP, "Phi_phi0": torch.stack([ones, 0 * ones]), "Phi_r0": torch.stack([0 * ones, ones])}[group]
            d2.Phiphi, d2.Phir = dw.Phiphi + e * v[0], dw.Phir + e * v[1]
            delta = torch.stack([d2.Phiphi - dw.Phiphi, d2.Phir - dw.Phir])
            pred = float(torch.sum(out["gPhi_knots"] * delta))
        elif group == "theta":
            d2.theta = tpl.theta + e
            pred = gsc[0] * (d2.theta - tpl.theta)
        elif group == "phi":
            d2.phi = tpl.phi + e
            pred = gsc[1] * (d2.phi - tpl.phi)
        else:
            d2.scale = tpl.scale * (1.0 + e)
            pred = gsc[2] * (d2.scale - tpl.scale)
        return d2, pred

    eps = {"amplitudes": 1e-4, "phases": 1e-5, "Phi_phi0": 1e-5, "Phi_r0": 1e-5, "theta": 1e-5, "phi": 1e-5,
           "scale": 1e-4}
    for group, e in eps.items():
        dplus, pplus = shifted(e, group)
        dminus, pminus = shifted(-e, group)
        num = (loss(dplus) - loss(dminus)) / (2 * e)
        ana = (pplus - pminus) / (2 * e)
        print(f"draw {k} {group}: central difference {num:.10e}, adjoint {ana:.10e}")
        assert abs(num - ana) <= 1e-5 * abs(ana), (k, group, num, ana)
    # the Phi_0 gradients are the sums of the phase-knot gradients (a common offset)
    gk = out["gPhi_knots"].cpu().numpy()
    for r in range(2):
        assert abs(gk[r].sum() - gsc[3 + r]) <= 1e-9 * np.abs(gk[r]).sum()


def test_vjp_bitwise_repeatable_on_split_units(ctx):
    """The adjoint's chunks go to whichever wave asks first, but every sum runs
    in a fixed order: two calls on draw 10 of the forward+adjoint workload
    (units split into many chunks, chunk size above the minimum) give the
    same bits, in both precisions."""
    w = _cfg5_draw(10)
    dev = ctx.device
    dw = fd.DeviceWaveform.from_workload(w, device=dev)
    rng = np.random.default_rng(5)
    g = rng.normal(size=(4, w.Nf))
    gp = torch.as_tensor(g[0] + 1j * g[1], device=dev)
    gc = torch.as_tensor(g[2] + 1j * g[3], device=dev)
    for prec in ("fp64", "mixed"):
        a = ctx.vjp_dev(dw, gp, gc, prec)
        b = ctx.vjp_dev(dw, gp, gc, prec)
        torch.cuda.synchronize()
        assert ctx.sync_flags() == 0
        for key in a:
            assert torch.equal(a[key], b[key]), (prec, key)
        assert bool(torch.isfinite(torch.view_as_real(a["gA_knots"])).all())

"""torch.autograd wrapper of the frequency-domain waveform and its HIP adjoint,
plus the Whittle log-likelihood of Eq. likelihood in torch.

    hp, hc = fdemri_waveform(ctx, static, A, Phiphi, Phir, theta, phi, scale)
    L = whittle_loglike(hp, hc, dp, dc, S, wts)
    L.backward()      # gradients w.r.t. A, Phiphi, Phir, theta, phi, scale

The forward is fdemri_waveform; the backward is fdemri_vjp (the forward terms
are recomputed on the GPU, the frequency splines are held fixed).
"""
from __future__ import annotations

import torch

from . import Context, DeviceWaveform


class WaveformStatic:
    """The inputs that are not differentiated: trajectory times and
    fundamental frequencies (they fix the roots t(f)), mode numbers and the
    frequency grid."""

    def __init__(self, t, Fphi, Fr, l, m, n, f, partners=True, prec="fp64", device="cuda"):
        dev = torch.device(device)
        self.t = torch.as_tensor(t, dtype=torch.float64, device=dev).contiguous()
        self.Fphi = torch.as_tensor(Fphi, dtype=torch.float64, device=dev).contiguous()
        self.Fr = torch.as_tensor(Fr, dtype=torch.float64, device=dev).contiguous()
        self.l = torch.as_tensor(l, dtype=torch.int32, device=dev).contiguous()
        self.m = torch.as_tensor(m, dtype=torch.int32, device=dev).contiguous()
        self.n = torch.as_tensor(n, dtype=torch.int32, device=dev).contiguous()
        self.f = torch.as_tensor(f, dtype=torch.float64, device=dev).contiguous()
        self.partners = partners
        self.prec = prec
        self.device = dev

    def desc_inputs(self, A, Phiphi, Phir, theta, phi, scale):
        dw = DeviceWaveform.__new__(DeviceWaveform)
        dw.t, dw.Fphi, dw.Fr = self.t, self.Fphi, self.Fr
        dw.Phiphi = Phiphi.detach().to(torch.float64).contiguous()
        dw.Phir = Phir.detach().to(torch.float64).contiguous()
        dw.l, dw.m, dw.n, dw.f = self.l, self.m, self.n, self.f
        dw.A = torch.view_as_real(A.detach().to(torch.complex128)).contiguous()
        dw.theta, dw.phi, dw.scale = float(theta), float(phi), float(scale)
        dw.partners, dw.device = self.partners, self.device
        dw.coeffs_given = False
        return dw


class FDEmriFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, lib_ctx: Context, static: WaveformStatic, A, Phiphi, Phir, theta, phi, scale):
        dw = static.desc_inputs(A, Phiphi, Phir, theta, phi, scale)
        hp, hc = lib_ctx.waveform_dev(dw, static.prec)
        fctx.lib_ctx, fctx.static, fctx.dw = lib_ctx, static, dw
        fctx.A_dtype = A.dtype
        return hp, hc

    @staticmethod
    def backward(fctx, g_hp, g_hc):
        lib_ctx, static, dw = fctx.lib_ctx, fctx.static, fctx.dw
        zeros = torch.zeros(dw.Nf, dtype=torch.complex128, device=dw.device)
        g_hp = zeros if g_hp is None else g_hp
        g_hc = zeros if g_hc is None else g_hc
        out = lib_ctx.vjp_dev(dw, g_hp, g_hc, static.prec, coef=False, knots=True)
        gs = out["g_scalars"]
        gA = out["gA_knots"].to(fctx.A_dtype)
        return (None, None, gA, out["gPhi_knots"][0], out["gPhi_knots"][1], gs[0], gs[1], gs[2])


def fdemri_waveform(lib_ctx, static, A, Phiphi, Phir, theta, phi, scale):
    """Differentiable h_+(f), h_x(f).  A: [Nm, K] complex; Phiphi, Phir: [K];
    theta, phi, scale: 0-d float64 tensors (or floats, not differentiated)."""
    dev = static.device
    as_t = lambda x: x if torch.is_tensor(x) else torch.tensor(float(x), dtype=torch.float64, device=dev)
    return FDEmriFn.apply(lib_ctx, static, A, Phiphi, Phir, as_t(theta), as_t(phi), as_t(scale))


def whittle_loglike(hp, hc, dp, dc, S, wts):
    """-1/2 sum_alpha <d - h | d - h>_alpha with <a|b> = 4 Re sum conj(a) b w / S
    (Eq. likelihood, Eq. innerprod); bins with w = 0 or S = inf carry no weight."""
    L = hp.real.new_zeros(())
    for h, d in ((hp, dp), (hc, dc)):
        r = d - h
        L = L - 2.0 * torch.sum(wts * (r.real ** 2 + r.imag ** 2) / S)
    return L

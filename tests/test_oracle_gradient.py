"""Pins of the oracle's gradient against directional central finite
differences of the oracle waveform (Richardson-extrapolated), and of the
knot-value chain rule against perturbed knots."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.gradient import coef_grad_to_knots, waveform_vjp, whittle_cotangent
from oracle.likelihood import grid_weights, whittle_loglike
from oracle.waveform import splines, voices_from_modes, waveform_voices


def small_workload():
    w = W.inspiral_20_modes()
    sel = np.array([2, 6, 9, 13])          # n = -3, 1, 4, 8
    w.l, w.m, w.n, w.A = w.l[sel], w.m[sel], w.n[sel], w.A[sel]
    w.f = w.f[::9]
    return w


def loss_from(w, sp, d, S, wts, theta=None, phi=None, scale=None):
    th = w.theta if theta is None else theta
    ph = w.phi if phi is None else phi
    sc = w.scale if scale is None else scale
    h = waveform_voices(w.traj, sp, voices_from_modes(w.l, w.m, w.n, th, ph, sc), w.f)
    return whittle_loglike(d, h, S, wts)


@pytest.fixture(scope="module")
def setup():
    w = small_workload()
    sp = splines(w.traj, w.A)
    h = waveform_voices(w.traj, sp, voices_from_modes(w.l, w.m, w.n, w.theta, w.phi, w.scale), w.f)
    S = W.psd_closed_form(w.f)
    wts = grid_weights(w.f)
    rng = np.random.default_rng(4)
    # data: the waveform at slightly different amplitudes plus noise
    n1, n2 = W.noise_draw(w.f, wts[1], 9)
    d = (1.1 * h[0] + 0.05 * np.abs(h[0]).max() * (n1 != 0) * rng.normal(size=w.Nf),
         0.95 * h[1] + 0.05 * np.abs(h[1]).max() * (n2 != 0) * rng.normal(size=w.Nf))
    g_p, g_c = whittle_cotangent(d, h, S, wts)
    grad = waveform_vjp(w, g_p, g_c)
    return w, sp, d, S, wts, grad


def richardson(fun, eps):
    d1 = (fun(eps) - fun(-eps)) / (2 * eps)
    d2 = (fun(eps / 2) - fun(-eps / 2)) / eps
    return (4 * d2 - d1) / 3


def test_amplitude_coefficient_gradient(setup):
    w, sp, d, S, wts, grad = setup
    rng = np.random.default_rng(1)
    dA = (rng.normal(size=sp["A"].shape) + 1j * rng.normal(size=sp["A"].shape)) * np.abs(sp["A"]).mean(axis=(1, 2), keepdims=True)

    def L(e):
        s2 = dict(sp)
        s2["A"] = sp["A"] + e * dA
        return loss_from(w, s2, d, S, wts)
    fd = richardson(L, 1e-3)
    # gA is ascending; scipy's coefficient arrays are highest power first
    dA_asc = np.transpose(dA[::-1], (2, 1, 0))
    an = float(np.sum(np.real(np.conj(grad["gA"]) * dA_asc)))
    assert abs(an - fd) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("key,row", [("Phiphi", 0), ("Phir", 1)])
def test_phase_coefficient_gradient(setup, key, row):
    w, sp, d, S, wts, grad = setup
    rng = np.random.default_rng(2)
    dP = rng.normal(size=sp[key].shape) * np.array([1e-18, 1e-13, 1e-8, 1e-3])[:, None]

    def L(e):
        s2 = dict(sp)
        s2[key] = sp[key] + e * dP
        return loss_from(w, s2, d, S, wts)
    fd = richardson(L, 1.0)
    an = float(np.sum(grad["gPhi"][row] * dP[::-1].T))
    assert abs(an - fd) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("idx,name", [(0, "theta"), (1, "phi"), (2, "scale")])
def test_scalar_gradients(setup, idx, name):
    w, sp, d, S, wts, grad = setup
    base = {"theta": w.theta, "phi": w.phi, "scale": w.scale}[name]
    eps = 1e-3 * (abs(base) if name == "scale" else 1.0)
    fd = richardson(lambda e: loss_from(w, sp, d, S, wts, **{name: base + e}), eps)
    assert abs(grad["g_scalars"][idx] - fd) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("key,idx", [("Phiphi", 3), ("Phir", 4)])
def test_initial_phase_gradients(setup, key, idx):
    w, sp, d, S, wts, grad = setup

    def L(e):
        s2 = dict(sp)
        s2[key] = sp[key].copy()
        s2[key][3] = sp[key][3] + e
        return loss_from(w, s2, d, S, wts)
    fd = richardson(L, 1e-3)
    assert abs(grad["g_scalars"][idx] - fd) <= 1e-6 * abs(fd)


def test_knot_chain_rule(setup):
    """Gradient w.r.t. amplitude knot values via the transposed spline map."""
    w, sp, d, S, wts, grad = setup
    gk = coef_grad_to_knots(w.traj.t, grad["gA"])          # (Nm, K) complex
    rng = np.random.default_rng(3)
    dY = (rng.normal(size=w.A.shape) + 1j * rng.normal(size=w.A.shape)) * np.abs(w.A)

    def L(e):
        s2 = splines(w.traj, w.A + e * dY)
        return loss_from(w, s2, d, S, wts)
    fd = richardson(L, 1e-3)
    an = float(np.sum(np.real(np.conj(gk) * dY)))
    assert abs(an - fd) <= 1e-6 * abs(fd)

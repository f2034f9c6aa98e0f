"""Pins of the oracle's inner product, Hann convolution and fused likelihood
sums (Eqs. innerprod and likelihood; the Hann window in the frequency domain
on the DFT grid) against identities that do not use their code: the DFT of a
windowed real series, Parseval's theorem, and the existing Whittle
log-likelihood."""
import numpy as np

from oracle.likelihood import fused_sums, grid_weights, inner_product, whittle_loglike
from oracle.td import fd_hann, td_spectrum


def test_fd_hann_is_the_transform_of_the_windowed_series():
    # x_w[n] = x[n] (1/2 - 1/2 cos(2 pi n / N)) transforms, bin by bin, into
    # X[k]/2 - X[k+1]/4 - X[k-1]/4 (exact DFT identity); fd_hann drops the
    # neighbour past the last bin, so the Nyquist bin is left out
    rng = np.random.default_rng(11)
    N, dt = 512, 3.0
    x = rng.standard_normal(N)
    lhs = td_spectrum(x, dt, window=True)
    rhs = fd_hann(td_spectrum(x, dt, window=False))
    k = np.arange(N // 2)
    assert np.max(np.abs(lhs[k] - rhs[k])) <= 1e-12 * np.max(np.abs(lhs))


def test_inner_product_parseval_white_noise():
    # a zero-mean real series with no Nyquist content: for a constant PSD S,
    # <x|x> = 4 sum_{k>=1} |x~_k|^2 (1/T) / S = (2/S) dt sum_n x_n^2
    rng = np.random.default_rng(5)
    N, dt, S0 = 1024, 0.5, 3.7
    n = np.arange(N)
    x = np.zeros(N)
    for k in range(1, N // 2):
        x += rng.standard_normal() * np.cos(2 * np.pi * k * n / N + rng.uniform(0, 2 * np.pi))
    xf = td_spectrum(x, dt, window=False)
    f = np.arange(xf.size) / (N * dt)
    w = grid_weights(f)
    lhs = inner_product(xf, xf, np.full(f.size, S0), w)
    rhs = 2.0 / S0 * dt * np.sum(x * x)
    assert abs(lhs - rhs) <= 1e-11 * rhs


def _case(seed, n=700):
    rng = np.random.default_rng(seed)
    f = np.arange(n) * 1e-4
    S = 1.0 + rng.uniform(size=n)
    S[0] = np.inf
    w = grid_weights(f)
    wS = np.where(np.isfinite(S), 4.0 * w / np.where(np.isfinite(S), S, 1.0), 0.0)
    d = [rng.normal(size=n) + 1j * rng.normal(size=n) for _ in range(2)]
    h = [rng.normal(size=n) + 1j * rng.normal(size=n) for _ in range(2)]
    return d, h, S, w, wS


def test_fused_sums_match_whittle_loglike_and_inner_products():
    d, h, S, w, wS = _case(2)
    ll, hh, dh = fused_sums(d, h, wS)
    assert abs(ll - whittle_loglike(d, h, S, w)) <= 1e-12 * abs(ll)
    assert abs(hh - sum(inner_product(a, a, S, w) for a in h)) <= 1e-12 * hh
    assert abs(dh - sum(inner_product(a, b, S, w) for a, b in zip(d, h))) <= 1e-12 * abs(dh)
    # the same with the Hann-convolved model
    llw, hhw, dhw = fused_sums(d, h, wS, hann=True)
    g = [fd_hann(a) for a in h]
    assert abs(llw - whittle_loglike(d, g, S, w)) <= 1e-12 * abs(llw)
    assert abs(hhw - sum(inner_product(a, a, S, w) for a in g)) <= 1e-12 * hhw


def test_fused_sums_vanish_on_the_model_and_scale():
    d, h, S, w, wS = _case(4)
    ll, hh, dh = fused_sums(h, h, wS)
    assert ll == 0.0 and abs(dh - hh) <= 1e-13 * hh
    # log L is quadratic in the residual
    ll1 = fused_sums(d, h, wS)[0]
    ll2 = fused_sums([2 * a - b for a, b in zip(d, h)], h, wS)[0]
    assert abs(ll2 - 4 * ll1) <= 1e-12 * abs(ll2)

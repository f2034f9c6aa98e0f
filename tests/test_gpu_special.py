"""The device factor of Eq. extendedspa1 on its own (fdemri_spa_factor, the
code the mode sum runs at every root) against the oracle's G, which is
pinned to mpmath's K_{1/3} and Airy functions (test_oracle_special.py).

|X| = 2 pi |Fd|^3 / (3 Fdd^2) spans [1e-6, 1e12] with both signs, wave by
wave (64 consecutive elements share the choice of the series length), plus
waves at the switches between the Airy tables and the large-argument series
(|X| = 40) and between the series lengths (|1/X| = 1e-3 and 1e-5), waves that
mix a large and a small |X| (the whole wave then takes the long series), a
root on a turning point (Fd = 0, both piece directions) and Fdd = 0.
Bars: FP64 1e-13 relative per element; FP32 5e-7 relative per element (the
factor is formed in FP32 from FP64 derivatives: a handful of FP32 roundings
in the reciprocal square root, the series or table and two products, each
at most 6e-8)."""
import math

import numpy as np
import pytest
import torch

from oracle.special import G as G_oracle

pytestmark = pytest.mark.gpu
fd = pytest.importorskip("paper_2307_12585_amd")


@pytest.fixture(scope="module")
def ctx():
    c = fd.Context(0)
    yield c
    c.close()


def derivs_for(X, rng):
    """(Fd, Fdd) with the given X: |Fd| log-uniform in [1e-13, 1e-6] Hz/s,
    sgn Fd = sgn X, Fdd of random sign with Fdd^2 = 2 pi |Fd|^3 / (3 |X|)."""
    X = np.asarray(X, np.float64)
    fd_ = np.sign(X) * 10.0 ** rng.uniform(-13, -6, X.size)
    fdd = np.sqrt(2 * math.pi * np.abs(fd_) ** 3 / (3 * np.abs(X))) * rng.choice([-1.0, 1.0], X.size)
    return fd_, fdd


def cases():
    rng = np.random.default_rng(8)
    waves = []
    for d in range(-6, 12):                      # one wave per decade and sign
        for sg in (1.0, -1.0):
            waves.append(sg * 10.0 ** rng.uniform(d, d + 1, 64))
    for xb in (40.0, 1e3, 1e5):                  # the switches, just below and above
        for side in (1 - 1e-9, 1 + 1e-9, 1 - 1e-3, 1 + 1e-3):
            waves.append(xb * side * rng.choice([-1.0, 1.0], 64))
    mix = np.where(np.arange(64) % 2 == 0, 1e9, 50.0) * rng.choice([-1.0, 1.0], 64)
    waves.append(mix)
    waves.append(np.where(np.arange(64) < 63, 2e4, 1e2))
    X = np.concatenate(waves)
    gd, gdd = derivs_for(X, rng)
    d = np.where(rng.uniform(size=X.size) < 0.5, -1, 1).astype(np.int32)
    # a root on a turning point (Fd = 0), both directions; Fdd = 0; Fd = Fdd = 0
    gd = np.concatenate([gd, np.zeros(64), 10.0 ** rng.uniform(-13, -6, 64) * rng.choice([-1.0, 1.0], 64), [0.0]])
    gdd = np.concatenate([gdd, 10.0 ** rng.uniform(-20, -14, 64) * rng.choice([-1.0, 1.0], 64), np.zeros(64), [0.0]])
    d = np.concatenate([d, np.tile(np.array([1, -1], np.int32), 32), np.ones(64, np.int32), [1]]).astype(np.int32)
    return gd, gdd, d


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("mixed", 5e-7)])
def test_device_factor_against_oracle(ctx, prec, tol):
    gd, gdd, d = cases()
    ref = G_oracle(gd, gdd, d)
    dev = ctx.device
    got = ctx.spa_factor(torch.as_tensor(gd, device=dev), torch.as_tensor(gdd, device=dev),
                         torch.as_tensor(d, device=dev), prec).cpu().numpy().astype(np.complex128)
    assert got[-1] == 0 and ref[-1] == 0
    err = np.abs(got[:-1] - ref[:-1]) / np.abs(ref[:-1])
    worst = int(np.argmax(err))
    with np.errstate(divide="ignore"):
        X = 2 * math.pi * gd[worst] ** 3 / (3 * gdd[worst] ** 2)
    print(f"{prec}: max rel error {err.max():.3e} at element {worst} (X = {X:.6g}), median {np.median(err):.3e}")
    assert err.max() <= tol


def test_invalid_arguments(ctx):
    with pytest.raises(fd.FdemriError):
        ctx._check(ctx._lib.fdemri_spa_factor(ctx._h, 0, -1, None, None, None, None, None))
    z = torch.zeros(0, dtype=torch.float64, device=ctx.device)
    assert ctx.spa_factor(z, z, z.to(torch.int32)).numel() == 0

"""fdemri_trajectory (through the C ABI): device trajectories against the
oracle's (SciPy DOP853 at a tighter tolerance) and against the closed forms of
the circular inspiral and the eccentric-orbit invariant; the knots then drive
the mode sum like host-made ones."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle.trajectory import G_MSUN_OVER_C3, peters_invariant, trajectory

pytestmark = pytest.mark.gpu
fd = pytest.importorskip("paper_2307_12585_amd")


@pytest.fixture(scope="module")
def ctx():
    c = fd.Context(0)
    yield c
    c.close()


CASES = [
    dict(M=1e6, mu=10.0, p0=12.0, e0=0.3, T=0.25 * W.YRSID_SI),      # the 20-mode source
    dict(M=2e6, mu=20.0, p0=13.0, e0=0.45, T=2.0 * W.YRSID_SI),      # the 3842-mode source
    dict(M=1e6, mu=30.0, p0=9.5, e0=0.4, T=5e7, Phiphi0=1.3, Phir0=-0.4),  # plunges
    dict(M=1e5, mu=50.0, p0=7.0, e0=0.0, T=1e9),                     # circular, plunges
    dict(M=3e5, mu=80.0, p0=15.0, e0=0.05, T=4.0 * W.YRSID_SI),
]


def test_trajectories_match_oracle(ctx):
    K = 100
    got = ctx.trajectory(CASES, K).cpu().numpy()
    assert ctx.sync_flags() == 0
    for P, g in zip(CASES, got):
        ref = trajectory(P["M"], P["mu"], P["p0"], P["e0"], P["T"], K, P.get("Phiphi0", 0.0), P.get("Phir0", 0.0))
        # end time (T or the located plunge), knot times
        assert abs(g[0][-1] - ref[0][-1]) <= 1e-9 * ref[0][-1], (P, g[0][-1], ref[0][-1])
        np.testing.assert_allclose(g[0], ref[0], rtol=1e-9, atol=0)
        # p, e, frequencies: the two integrators' tolerances (1e-12 and 1e-13)
        for row in (1, 2, 5):
            np.testing.assert_allclose(g[row], ref[row], rtol=2e-9)
        np.testing.assert_allclose(g[6], ref[6], rtol=2e-9, atol=1e-13)
        # phases: absolute error relative to the accumulated phase
        for row in (3, 4):
            assert np.max(np.abs(g[row] - ref[row])) <= 1e-9 * np.max(np.abs(ref[row])) + 1e-8


def test_circular_closed_form_and_invariant(ctx):
    P = dict(M=1e6, mu=10.0, p0=12.0, e0=0.0, T=1e7)
    g = ctx.trajectory([P], 64).cpu().numpy()[0]
    Ms, q = P["M"] * G_MSUN_OVER_C3, P["mu"] / P["M"]
    a = 256.0 / 5.0 * q / Ms
    p = (P["p0"] ** 4 - a * g[0]) ** 0.25
    assert np.max(np.abs(g[5] / p - 1)) <= 1e-11
    phi = 8.0 * (P["p0"] ** 2.5 - p ** 2.5) / (5.0 * a * Ms)
    assert np.max(np.abs(g[3][1:] / phi[1:] - 1)) <= 1e-10
    # eccentric: the invariant along the device trajectory
    e = ctx.trajectory([CASES[2]], 80).cpu().numpy()[0]
    inv = peters_invariant(e[5], e[6])
    assert np.max(np.abs(inv / inv[0] - 1)) <= 1e-10
    assert abs(e[5][-1] - (6 + 2 * e[6][-1] + 0.1)) <= 1e-9


def test_device_knots_drive_the_mode_sum(ctx):
    """The 20-mode source with device-made knots: the FD waveform equals the
    one from host knots to the level the knots agree (the phase differences
    of ~1e-9 of the accumulated phase)."""
    w = W.inspiral_20_modes()
    K = w.traj.t.size
    g = ctx.trajectory([CASES[0]], K)
    dw_host = fd.DeviceWaveform.from_workload(w, device=ctx.device)
    hp0, hc0 = ctx.waveform_dev(dw_host)
    desc = dw_host  # same modes, amplitudes, angles and grid; knots replaced below
    tr = g[0]
    dw = fd.DeviceWaveform(tr[0], tr[1], tr[2], tr[3], tr[4], w.l, w.m, w.n, w.A, w.theta, w.phi, w.scale, w.f,
                           device=ctx.device)
    hp1, hc1 = ctx.waveform_dev(dw)
    torch.cuda.synchronize()
    rel = float(torch.linalg.vector_norm(hp1 - hp0) / torch.linalg.vector_norm(hp0))
    print("waveform difference from host knots", rel)
    assert rel <= 1e-8

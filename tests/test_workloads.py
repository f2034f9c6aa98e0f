"""The synthetic input generators reproduce the paper's grid sizes and the
stated workload shapes."""
import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_grid_sizes.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_paper_full_grid_size():
    """Table tab:timing_source: T = 4 yr at dt = 10 s gives N_f = 6311631 and
    N = 12623260 time samples with a sidereal year and N_t = round(T/dt)."""
    g = _golden()
    T = g["T_years"] * W.YRSID_SI
    f = W.rfft_grid(T, g["dt_s"])
    assert int(round(T / g["dt_s"])) == int(g["N_t_samples"])
    # the printed N_f counts the bins k = 0..N/2 of the real DFT
    assert f.size == int(g["N_f_full"])


def test_20_mode_workload_shapes():
    w = W.inspiral_20_modes()
    assert (w.K, w.Nm, w.Nf) == (100, 20, 394478)
    assert abs(w.traj.p[0] - 12.0) < 1e-12 and 11.8 < w.traj.p[-1] < 11.9
    assert np.all(np.diff(w.traj.t) > 0) and np.all(np.diff(w.f) > 0)


def test_3842_mode_workload_shapes():
    w = W.inspiral_3842_modes()
    assert w.K == 200 and w.Nf == 3155816
    assert 3800 <= w.Nm <= W.count_total_modes() == 3843
    assert np.all(w.m >= 0) and np.all(w.m <= w.l)


def test_log_grid_workload():
    w = W.inspiral_20_modes_log_grid()
    assert w.Nf == 10000 and abs(w.f[0] - 1e-4) < 1e-18 and abs(w.f[-1] - 0.1) < 1e-15


def test_batch_draws_reproducible():
    a = W.batch_params(3, 7)
    b = W.batch_params(3, 7)
    assert a == b
    w = W.batch_workload(a[0])
    assert w.A.shape == (w.Nm, w.K)


def test_noise_normalisation():
    """E<n|n> = 2 per bin (sum over N/2 bins = N), Sec. 2.3."""
    f = np.arange(1, 200001) * 1e-6
    df = 1e-6
    n1, n2 = W.noise_draw(f, df, 3)
    S = W.psd_closed_form(f)
    ip = 4 * np.sum(np.abs(n1) ** 2 / S) * df
    assert abs(ip / f.size - 2.0) < 0.03

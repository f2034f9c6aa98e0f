"""Pins of the oracle's frequency-domain mode sum (Sec. 2.2) against exact
Fourier transforms, the symmetries of Eq. main_wave, invariants of the
transform, and a windowed DFT of the time-domain voice sum (Sec. 2.3)."""
import math

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.harmonics import swsh
from oracle.likelihood import grid_weights
from oracle.td import fd_hann, mismatch, td_spectrum, td_waveform
from oracle.waveform import Voice, splines, waveform_voices


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _y22(w):
    return complex(swsh(-2, 2, 2, w.theta, w.phi))


# --- P1: linear chirp, exact Fresnel transform -----------------------------

@pytest.mark.parametrize("f0,fdot", [(1e-4, 1e-9), (2e-4, -1e-9)])
def test_linear_chirp_closed_form(f0, fdot):
    """F(t) = f0 + fdot t, quadratic phase, constant amplitude: the
    infinite-line transform is H |fdot|^{-1/2} e^{i[pi (f-f0)^2/fdot - Phi0 - pi/4 sgn fdot]}
    inside the swept band and the method gives 0 outside it."""
    A0, Phi0, T = 1.3 - 0.4j, 0.7, 1e5
    w = W.linear_chirp_workload(f0=f0, fdot=fdot, T=T, A0=A0, Phi0=Phi0, Nf=3001)
    _, _, hpos, hneg = oracle.waveform(w, partners=False, return_sides=True)
    H = w.scale * A0 * _y22(w)
    f = w.f
    tf = (f - f0) / fdot
    inside = (tf >= 0) & (tf <= T)
    ref = np.where(inside, H * abs(fdot) ** -0.5
                   * np.exp(1j * (math.pi * (f - f0) ** 2 / fdot - Phi0 - 0.25 * math.pi * np.sign(fdot))), 0)
    assert inside.sum() > 2000 and (~inside).sum() > 100
    assert rel_l2(hpos, ref) <= 1e-13
    assert np.all(hneg == 0)


def chirp_ft(H, f0, fdot, Phi0, T, nu):
    """Exact Fresnel transform at frequency nu (either sign) of the voice
    H e^{-i Phi(t)}, Phi = Phi0 + 2 pi (f0 t + fdot t^2/2), on the infinite
    line, kept where the stationary time (nu - f0)/fdot lies in [0, T] (the
    method's hard edge)."""
    tn = (nu - f0) / fdot
    val = H * abs(fdot) ** -0.5 * np.exp(1j * (math.pi * (nu - f0) ** 2 / fdot - Phi0
                                               - 0.25 * math.pi * np.sign(fdot)))
    return np.where((tn >= 0) & (tn <= T), val, 0)


def zero_crossing_workload(fdot, at_knot, T=1e5, K=40, Nf=3001):
    """A (2,2,0) voice whose frequency F_V = f0 + fdot t passes through zero
    inside the trajectory.  at_knot: the crossing falls exactly on knot 16
    (F_V there is exactly 0); otherwise f0 puts it between knots."""
    t = np.linspace(0.0, T, K)
    f0 = -fdot * t[16] if at_knot else -fdot * 0.4123 * T
    return W.linear_chirp_workload(f0=f0, fdot=fdot, T=T, K=K, Nf=Nf), f0


@pytest.mark.parametrize("fdot", [1e-9, -1e-9])
@pytest.mark.parametrize("at_knot", [False, True])
def test_zero_crossing_chirp_closed_form(fdot, at_knot):
    """F_V = f0 + fdot t changes sign (Sec. 2.2: all roots of F_V(t) = +-f;
    reading R5): the method cuts the voice at the crossing; the part with
    F_V < 0 feeds h(-f) and the part with F_V > 0 feeds h(+f).  Each side
    must equal the exact Fresnel transform at +f and -f respectively, which
    fixes the side chosen on each piece, the piece end 0 at the crossing, and
    the phase 2 pi (-f) t - Phi on the negative side."""
    A0, Phi0, T = 1.3 - 0.4j, 0.7, 1e5
    w, f0 = zero_crossing_workload(fdot, at_knot)
    if at_knot:
        assert 2 * w.traj.Fphi[16] == 0.0
    _, _, hpos, hneg = oracle.waveform(w, partners=False, return_sides=True)
    H = w.scale * A0 * _y22(w)
    f = w.f
    ref_pos = chirp_ft(H, f0, fdot, Phi0, T, f)
    ref_neg = chirp_ft(H, f0, fdot, Phi0, T, -f)
    # both sides carry a few hundred bins, and a bin band where only one does
    assert np.count_nonzero(ref_pos) > 500 and np.count_nonzero(ref_neg) > 500
    assert rel_l2(hpos, ref_pos) <= 1e-13
    assert rel_l2(hneg, ref_neg) <= 1e-13
    assert np.array_equal(hpos != 0, ref_pos != 0) and np.array_equal(hneg != 0, ref_neg != 0)


def test_zero_crossing_chirp_with_partner_polarizations():
    """The same crossing with the (2,-2,0) partner (H' = scale (-1)^l conj(A0)
    Y_{2,-2}, Phi' = -Phi_V): the partner's transform at nu is
    conj of the voice's transform at -nu with H -> conj H', and O7 combines
    both sides into h_+ and h_x.  Closed form against the oracle's
    polarizations."""
    A0, Phi0, T, fdot = 1.3 - 0.4j, 0.7, 1e5, 1e-9
    w, f0 = zero_crossing_workload(fdot, False)
    hp, hc = oracle.waveform(w, partners=True)
    f = w.f
    H = w.scale * A0 * _y22(w)
    Hp = w.scale * (-1) ** 2 * np.conj(A0) * complex(swsh(-2, 2, -2, w.theta, w.phi))
    pos = chirp_ft(H, f0, fdot, Phi0, T, f) + np.conj(chirp_ft(np.conj(Hp), f0, fdot, Phi0, T, -f))
    neg = chirp_ft(H, f0, fdot, Phi0, T, -f) + np.conj(chirp_ft(np.conj(Hp), f0, fdot, Phi0, T, f))
    ref_p = 0.5 * (pos + np.conj(neg))
    ref_c = 0.5j * (pos - np.conj(neg))
    assert rel_l2(hp, ref_p) <= 1e-13 and rel_l2(hc, ref_c) <= 1e-13


# --- P2: quadratic frequency (turnover), exact Airy transform ---------------

def turnover_workload(Fc, Fdd, Tc=1e4, K=41, Phic=0.3, A0=0.8 + 0.5j, Nf=3000):
    t = np.linspace(-Tc, Tc, K)
    F = Fc + 0.5 * Fdd * t * t
    Phi = Phic + 2 * math.pi * Fc * t + (math.pi / 3) * Fdd * t ** 3
    traj = W.Trajectory(t=t, Fphi=0.5 * F, Fr=np.zeros(K), Phiphi=0.5 * Phi, Phir=np.zeros(K),
                        p=np.full(K, 10.0), e=np.zeros(K))
    Fend = Fc + 0.5 * Fdd * Tc * Tc
    lo, hi = sorted((Fc, Fend))
    f = np.linspace(lo, hi, Nf + 2)[1:-1]
    return W.Workload(traj=traj, l=np.array([2], np.int32), m=np.array([2], np.int32),
                      n=np.array([0], np.int32), A=np.full((1, K), A0), theta=1.1, phi=0.2,
                      scale=1.0, f=f)


@pytest.mark.parametrize("K", [41, 40])
@pytest.mark.parametrize("Fc,Fdd", [(1e-2, 1e-9), (6e-2, -1e-9)])
def test_turnover_two_roots_equal_airy_transform(Fc, Fdd, K):
    """F = Fc + Fdd (t-tc)^2/2 with cubic phase: the exact transform is
    H 2 pi (pi|Fdd|)^{-1/3} Ai(-sgn(Fdd) 2 pi (f-Fc) (pi|Fdd|)^{-1/3}) e^{i(2 pi f tc - Phi_c)},
    and the method's sum over the two roots reproduces it on the side where
    both roots exist (this fixes the sign of Eq. extendedspa1 and exercises
    the special function from X ~ 0 to X ~ 1e3).  K = 41 puts the turnover
    exactly on a knot (t = 0), K = 40 inside a segment."""
    w = turnover_workload(Fc, Fdd, K=K)
    assert (0.0 in w.traj.t) == (K == 41)
    _, _, hpos, _ = oracle.waveform(w, partners=False, return_sides=True)
    H = w.scale * w.A[0, 0] * _y22(w)
    c = (math.pi * abs(Fdd)) ** (-1 / 3)
    mpmath.mp.dps = 30
    ref = np.array([complex(H * 2 * mpmath.pi * c
                            * mpmath.airyai(-np.sign(Fdd) * 2 * mpmath.pi * (mpmath.mpf(fk) - Fc) * c)
                            * mpmath.exp(-1j * mpmath.mpf(0.3))) for fk in w.f])
    assert rel_l2(hpos, ref) <= 1e-12
    # the sum over roots is needed: one root alone is far off
    assert np.max(np.abs(hpos)) > 0


# --- P4: partner voices ------------------------------------------------------

def test_partner_identity():
    """h_{l,-m,-n}(-f) = conj( h_{l,m,n}(f) with H -> conj H' ), where
    H' = scale (-1)^l conj(A) Y_{l,-m}: the negative-frequency branch of the
    explicit partner equals the conjugate of the positive branch."""
    w = W.inspiral_20_modes()
    sp = splines(w.traj, w.A)
    f = w.f[::7]
    for mu in [0, 4, 11]:
        l, m, n = int(w.l[mu]), int(w.m[mu]), int(w.n[mu])
        yp = complex(swsh(-2, l, -m, w.theta, w.phi))
        partner = Voice(-m, -n, mu, True, w.scale * (-1) ** l * yp)
        mirrored = Voice(m, n, mu, False, np.conj(w.scale * (-1) ** l * yp) * 1.0)
        _, _, pos_p, neg_p = waveform_voices(w.traj, sp, [partner], f, return_sides=True)
        _, _, pos_m, neg_m = waveform_voices(w.traj, sp, [mirrored], f, return_sides=True)
        assert np.allclose(neg_p, np.conj(pos_m), rtol=0, atol=1e-15 * np.abs(pos_m).max())
        assert np.allclose(pos_p, np.conj(neg_m), rtol=0, atol=1e-15 * max(np.abs(neg_m).max(), 1e-300))
        assert np.abs(neg_p).max() + np.abs(pos_p).max() > 0


# --- P5: polarization ratio of a single (2,2,n) mode ------------------------

def test_polarization_ratio_single_22_mode():
    """For one (2,2,n) mode with F > 0 throughout, h_x/h_+ = 2i cos(theta)/(1+cos^2 theta)."""
    w = W.inspiral_20_modes()
    sel = np.nonzero(w.n == 3)[0]
    w.l, w.m, w.n, w.A = w.l[sel], w.m[sel], w.n[sel], w.A[sel]
    hp, hc = oracle.waveform(w)
    nz = np.abs(hp) > 0
    assert nz.sum() > 300
    ratio = hc[nz] / hp[nz]
    ct = math.cos(w.theta)
    assert np.allclose(ratio, 2j * ct / (1 + ct * ct), rtol=1e-13, atol=0)


# --- P6: invariants -----------------------------------------------------------

def _small_cfg1():
    w = W.inspiral_20_modes()
    w.f = w.f[::3]
    return w


def test_time_shift_invariant():
    w = _small_cfg1()
    hp, hc = oracle.waveform(w)
    d = 1234.5
    w.traj.t = w.traj.t + d
    hp2, hc2 = oracle.waveform(w)
    ph = np.exp(2j * math.pi * w.f * d)
    assert rel_l2(hp2, hp * ph) <= 1e-10 and rel_l2(hc2, hc * ph) <= 1e-10


def test_linearity_in_amplitude_and_scale():
    w = _small_cfg1()
    hp1, hc1 = oracle.waveform(w)
    A1 = w.A.copy()
    rng = np.random.default_rng(5)
    A2 = A1 * (rng.normal(size=A1.shape[0]) + 1j)[:, None]
    w.A = A2
    hp2, hc2 = oracle.waveform(w)
    # real-linear (partners carry conj A): real coefficients only
    w.A = 2.0 * A1 - 3.0 * A2
    w.scale *= 1.5
    hp3, hc3 = oracle.waveform(w)
    assert rel_l2(hp3, 1.5 * (2 * hp1 - 3 * hp2)) <= 1e-13
    assert rel_l2(hc3, 1.5 * (2 * hc1 - 3 * hc2)) <= 1e-13


def test_phase_offset_invariant():
    """Adding delta to Phi_phi multiplies each voice by e^{-i m_V delta}: with
    only (2,2,n>=0) modes (F_V > 0), h(+f) turns by e^{-2i delta} and the
    partners' h(-f) by e^{+2i delta}."""
    w = _small_cfg1()
    sel = w.n >= 0
    w.l, w.m, w.n, w.A = w.l[sel], w.m[sel], w.n[sel], w.A[sel]
    hp, hc, hpos, hneg = oracle.waveform(w, return_sides=True)
    delta = 0.4321
    w.traj.Phiphi = w.traj.Phiphi + delta
    _, _, hpos2, hneg2 = oracle.waveform(w, return_sides=True)
    # the shifted knot phases (up to ~1e5 rad) are re-rounded: ~m ulp(Phi)
    tol = 8 * np.spacing(np.abs(w.traj.Phiphi).max())
    assert rel_l2(hpos2, hpos * np.exp(-2j * delta)) <= tol
    assert rel_l2(hneg2, hneg * np.exp(2j * delta)) <= tol


def test_dc_bin_zero_and_evals_count():
    w = W.inspiral_20_modes()
    hp, hc = oracle.waveform(w, f=w.f[:2000])
    assert hp[0] == 0 and hc[0] == 0
    assert oracle.waveform.__module__ == "oracle.waveform"
    from oracle.waveform import count_evals
    assert count_evals(w) == 8724


# --- P7: against the windowed DFT of the time-domain sum --------------------

def test_spa_against_windowed_dft():
    """Mismatch between the FD waveform (Hann-convolved) and the DFT of the
    Hann-windowed TD voice sum from the same splines is <= 1e-3 (Sec. 2.3)."""
    Nt, dt = 2 ** 17, 5.0
    T = Nt * dt
    traj = W.peters_trajectory(1e5, 10, 12, 0.2, T, 100)
    n = np.arange(-2, 5, dtype=np.int32)
    rng = np.random.default_rng(3)
    A = (0.2 ** np.abs(n) * np.exp(1j * rng.uniform(0, 2 * np.pi, 7)))[:, None] * (traj.p / 12)[None, :] ** -1
    f = np.arange(Nt // 2 + 1) / T
    w = W.Workload(traj=traj, l=np.full(7, 2, np.int32), m=np.full(7, 2, np.int32), n=n, A=A,
                   theta=0.8, phi=0.3, scale=1.0, f=f)
    hp, hc = oracle.waveform(w)
    h = td_waveform(w, np.arange(Nt) * dt)
    tp, tc = td_spectrum(h.real, dt), td_spectrum(-h.imag, dt)
    S = W.psd_closed_form(f)
    wt = grid_weights(f)
    wt[-1] = 0
    mm = mismatch((fd_hann(hp), fd_hann(hc)), (tp, tc), S, wt)
    assert 0 <= mm <= 1e-3
    # a sign error anywhere (e.g. the constant of Eq. extendedspa1) is caught
    assert mismatch((fd_hann(-hp), fd_hann(-hc)), (tp, tc), S, wt) > 1.0

"""Seeded synthetic inputs for the frequency-domain EMRI mode sum.

This module produces *inputs* only: sparse inspiral trajectories, per-mode
amplitude knot values, frequency grids, a noise spectral density and noise
draws.  It holds none of the waveform method's arithmetic (no splines, no
stationary-phase evaluation, no spin-weighted harmonics), so that both the
CPU oracle and the HIP library can consume the same inputs without sharing
any code of the method.

The paper's own workloads need precomputed flux and Teukolsky-amplitude data
(Sec. 2.1) that are not available; these generators stand in for them with
the same shapes: ~100-200 knot trajectories from an adaptive integrator
(Sec. 2.1), up to 3843 (l,m,n) modes, full rfft frequency grids of millions
of bins (Sec. 2.3, Table tab:timing_source) and downsampled grids (Sec. 3.3).

Trajectory model: Peters-type orbit-averaged fluxes for (p, e) with the toy
fundamental frequencies Omega_phi = p^-3/2 (1-e^2)^3/2 and
Omega_r = Omega_phi sqrt(1 - 6/p), phases Phi = integral of Omega / M
(the ODE system of Sec. 2.1 with synthetic fluxes).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
from scipy.integrate import solve_ivp

# Physical constants (SI / geometric).
MTSUN_SI = 4.925490947641267e-6      # G Msun / c^3 [s]
MRSUN_SI = 1476.6250385063           # G Msun / c^2 [m]
GPC_SI = 3.0856775814913673e25       # 1 Gpc [m]
YRSID_SI = 31558149.763545603        # sidereal year [s]

__all__ = [
    "MTSUN_SI", "MRSUN_SI", "GPC_SI", "YRSID_SI",
    "Trajectory", "Workload", "peters_trajectory", "mode_table",
    "rfft_grid", "log_grid", "inspiral_20_modes", "inspiral_3842_modes", "inspiral_20_modes_log_grid",
    "batch_params", "batch_workload", "psd_closed_form", "noise_draw",
    "linear_chirp_workload", "count_total_modes",
]


@dataclass
class Trajectory:
    """Sparse trajectory knots (Sec. 2.1): times and the fundamental
    frequencies / phases of the Schwarzschild toy model."""
    t: np.ndarray        # [K] s, strictly increasing, t[0] = 0
    Fphi: np.ndarray     # [K] Hz = Omega_phi / (2 pi M_s)
    Fr: np.ndarray       # [K] Hz = Omega_r / (2 pi M_s)
    Phiphi: np.ndarray   # [K] rad, includes Phi_phi0
    Phir: np.ndarray     # [K] rad, includes Phi_r0
    p: np.ndarray        # [K] semi-latus rectum (M)
    e: np.ndarray        # [K] eccentricity


@dataclass
class Workload:
    """Everything one waveform evaluation needs, in the paper's terms:
    trajectory knots, mode numbers and complex amplitude knot values,
    viewing angles, the mu/d_L scale and the frequency array."""
    traj: Trajectory
    l: np.ndarray        # [Nm] int32
    m: np.ndarray        # [Nm] int32, 0 <= m <= l
    n: np.ndarray        # [Nm] int32
    A: np.ndarray        # [Nm, K] complex128 amplitude knot values
    theta: float
    phi: float
    scale: float         # mu / d_L (dimensionless)
    f: np.ndarray        # [Nf] Hz ascending, f >= 0
    meta: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return int(self.traj.t.size)

    @property
    def Nm(self) -> int:
        return int(self.l.size)

    @property
    def Nf(self) -> int:
        return int(self.f.size)


def _omegas(p, e):
    om_phi = p ** -1.5 * (1.0 - e * e) ** 1.5
    om_r = om_phi * np.sqrt(1.0 - 6.0 / p)
    return om_phi, om_r


def peters_trajectory(M: float, mu: float, p0: float, e0: float, T: float,
                      K: int, Phiphi0: float = 0.0, Phir0: float = 0.0) -> Trajectory:
    """Integrate the toy inspiral (DOP853, rtol 1e-12) from t=0 until T seconds
    or until p reaches 6 + 2e + 0.1, then sample K knots uniformly in time."""
    Ms = M * MTSUN_SI
    q = mu / M

    def rhs(_t, y):
        p, e = y[0], y[1]
        one_e2 = 1.0 - e * e
        dp = -(64.0 / 5.0) * q * one_e2 ** 1.5 * p ** -3 * (1.0 + 7.0 * e * e / 8.0) / Ms
        de = -(304.0 / 15.0) * q * e * one_e2 ** 1.5 * p ** -4 * (1.0 + 121.0 * e * e / 304.0) / Ms
        om_phi, om_r = _omegas(p, e)
        return [dp, de, om_phi / Ms, om_r / Ms]

    def plunge(_t, y):
        return y[0] - (6.0 + 2.0 * y[1] + 0.1)
    plunge.terminal = True
    plunge.direction = -1

    sol = solve_ivp(rhs, (0.0, T), [p0, e0, Phiphi0, Phir0], method="DOP853",
                    rtol=1e-12, atol=[1e-12, 1e-14, 1e-9, 1e-9], dense_output=True,
                    events=plunge)
    t_end = float(sol.t[-1])
    t = np.linspace(0.0, t_end, K)
    y = sol.sol(t)
    p, e = y[0], y[1]
    om_phi, om_r = _omegas(p, e)
    two_pi_Ms = 2.0 * math.pi * Ms
    return Trajectory(t=t, Fphi=om_phi / two_pi_Ms, Fr=om_r / two_pi_Ms,
                      Phiphi=y[2].copy(), Phir=y[3].copy(), p=p.copy(), e=e.copy())


def mode_table(lmax: int = 10, nmax: int = 30):
    """(l, m, n) table with l = 2..lmax, m = 0..l, n = -nmax..nmax, in
    l-ascending, then m, then n order (3843 modes for lmax=10, nmax=30)."""
    ls, ms, ns = [], [], []
    for l in range(2, lmax + 1):
        for m in range(0, l + 1):
            for n in range(-nmax, nmax + 1):
                ls.append(l); ms.append(m); ns.append(n)
    return (np.asarray(ls, np.int32), np.asarray(ms, np.int32), np.asarray(ns, np.int32))


def count_total_modes(lmax: int = 10, nmax: int = 30) -> int:
    return sum(l + 1 for l in range(2, lmax + 1)) * (2 * nmax + 1)


def rfft_grid(T: float, dt: float) -> np.ndarray:
    """Full DFT grid f_k = k / (N_t dt), k = 0..N_t//2, with N_t = round(T/dt)."""
    Nt = int(round(T / dt))
    return np.arange(Nt // 2 + 1, dtype=np.float64) / (Nt * dt)


def log_grid(fmin: float, fmax: float, N: int) -> np.ndarray:
    return np.geomspace(fmin, fmax, N)


def _scale(mu: float, dL_gpc: float = 1.0) -> float:
    return mu * MRSUN_SI / (dL_gpc * GPC_SI)


def _select(power: np.ndarray, eps: float) -> np.ndarray:
    """Keep modes whose power exceeds eps of the total.  The synthetic
    amplitude law has a time factor common to all modes, so the per-knot
    selection is the same at every knot and the union over knots is this."""
    return power > eps * power.sum()


def inspiral_20_modes(seed: int = 0, K: int = 100) -> Workload:
    """Small single waveform: M=1e6, mu=10, p0=12, e0=0.3, T=0.25 yr at
    dt=10 s on the full rfft grid; 20 modes l=2, m=2, n=-5..14 with
    A = a_n (p/p0)^-1 e^{i phi_n}, a_n = e0^|n| LN(0, 0.3), phi_n ~ U[0, 2pi)."""
    M, mu, p0, e0 = 1e6, 10.0, 12.0, 0.3
    T = 0.25 * YRSID_SI
    dt = 10.0
    rng = np.random.default_rng(seed)
    traj = peters_trajectory(M, mu, p0, e0, T, K)
    n = np.arange(-5, 15, dtype=np.int32)
    l = np.full(n.size, 2, np.int32)
    m = np.full(n.size, 2, np.int32)
    a = e0 ** np.abs(n) * rng.lognormal(0.0, 0.3, n.size)
    ph = rng.uniform(0.0, 2 * math.pi, n.size)
    A = (a * np.exp(1j * ph))[:, None] * (traj.p / p0)[None, :] ** -1
    return Workload(traj=traj, l=l, m=m, n=n, A=A, theta=math.pi / 3, phi=math.pi / 4,
                    scale=_scale(mu), f=rfft_grid(T, dt),
                    meta=dict(name="inspiral_20_modes", M=M, mu=mu, p0=p0, e0=e0, T=T, dt=dt, seed=seed))


def _law_amplitudes(rng, e0: float, l, m, n, p, p0):
    """Calibrated synthetic law |a|^2 = (1+|n|)^(-0.35/e0) LN(0,0.3)^2 with
    uniform phase; all lognormals first (table order), then all phases."""
    ln = rng.lognormal(0.0, 0.3, l.size)
    ph = rng.uniform(0.0, 2 * math.pi, l.size)
    a = (1.0 + np.abs(n)) ** (-0.175 / e0) * ln
    return a * np.exp(1j * ph), a * a


def inspiral_3842_modes(seed: int = 0, K: int = 200, eps: float = 1e-5) -> Workload:
    """Realistic single waveform: M=2e6, mu=20, p0=13, e0=0.45, T=2 yr at
    dt=10 s, K=200 knots, l=2..10, m=0..l, n=-30..30 selected at 1e-5 of the
    total power."""
    M, mu, p0, e0 = 2e6, 20.0, 13.0, 0.45
    T = 2.0 * YRSID_SI
    dt = 10.0
    rng = np.random.default_rng(seed)
    traj = peters_trajectory(M, mu, p0, e0, T, K)
    l, m, n = mode_table()
    a, power = _law_amplitudes(rng, e0, l, m, n, traj.p, p0)
    keep = _select(power, eps)
    A = a[keep][:, None] * (traj.p / p0)[None, :] ** -1
    return Workload(traj=traj, l=l[keep], m=m[keep], n=n[keep], A=A,
                    theta=math.pi / 3, phi=math.pi / 4, scale=_scale(mu), f=rfft_grid(T, dt),
                    meta=dict(name="inspiral_3842_modes", M=M, mu=mu, p0=p0, e0=e0, T=T, dt=dt, seed=seed))


def inspiral_20_modes_log_grid(seed: int = 0) -> Workload:
    """Config 1 evaluated on 1e4 log-spaced frequencies in [1e-4, 1e-1] Hz."""
    w = inspiral_20_modes(seed)
    w.f = log_grid(1e-4, 1e-1, 10_000)
    w.meta["name"] = "inspiral_20_modes_log_grid"
    return w


def batch_params(count: int, seed: int):
    """Draws for the batched workloads: M log-U[1e5,1e7], mu U[1,100],
    e0 U[0.05,0.5], p0 U[10,16], T U[0.5,4] yr, Phi0 U[0,2pi)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        out.append(dict(M=float(10 ** rng.uniform(5, 7)), mu=float(rng.uniform(1, 100)),
                        e0=float(rng.uniform(0.05, 0.5)), p0=float(rng.uniform(10, 16)),
                        T=float(rng.uniform(0.5, 4.0) * YRSID_SI),
                        Phiphi0=float(rng.uniform(0, 2 * math.pi)),
                        Phir0=float(rng.uniform(0, 2 * math.pi)),
                        seed=int(rng.integers(0, 2 ** 31 - 1))))
    return out


def batch_workload(prm: dict, K: int = 100, dt: float = 10.0, eps: float = 1e-5,
                   f: np.ndarray | None = None) -> Workload:
    """One waveform of the batched distribution (synthetic law, 1e-5 power
    threshold, full rfft grid of its own duration unless f is given)."""
    rng = np.random.default_rng(prm["seed"])
    traj = peters_trajectory(prm["M"], prm["mu"], prm["p0"], prm["e0"], prm["T"], K,
                             prm["Phiphi0"], prm["Phir0"])
    l, m, n = mode_table()
    a, power = _law_amplitudes(rng, prm["e0"], l, m, n, traj.p, prm["p0"])
    keep = _select(power, eps)
    A = a[keep][:, None] * (traj.p / prm["p0"])[None, :] ** -1
    return Workload(traj=traj, l=l[keep], m=m[keep], n=n[keep], A=A,
                    theta=math.pi / 3, phi=math.pi / 4, scale=_scale(prm["mu"]),
                    f=rfft_grid(prm["T"], dt) if f is None else f,
                    meta=dict(name="batch", dt=dt, **prm))


def psd_closed_form(f: np.ndarray) -> np.ndarray:
    """Smooth one-sided PSD S(f) = (1e-41/f^2 + 1e-40)(1 + (f/0.025)^2);
    +inf at f = 0 so that the DC bin carries no weight."""
    f = np.asarray(f, np.float64)
    with np.errstate(divide="ignore"):
        s = (1e-41 / (f * f) + 1e-40) * (1.0 + (f / 0.025) ** 2)
    return s


def noise_draw(f: np.ndarray, df: float, seed: int):
    """Complex Gaussian noise per channel with Re, Im ~ N(0, S/(4 df)), so
    that the expected noise inner product per bin is 2 (sum over bins = N)."""
    rng = np.random.default_rng(seed)
    S = psd_closed_form(f)
    sig = np.sqrt(np.where(np.isfinite(S), S, 0.0) / (4.0 * df))
    out = []
    for _ in range(2):
        out.append(sig * (rng.standard_normal(f.size) + 1j * rng.standard_normal(f.size)))
    return out[0], out[1]


def linear_chirp_workload(f0=2e-3, fdot=1e-10, T=2e6, K=40, A0=1.3 - 0.4j,
                          Phi0=0.7, Nf=4000, theta=0.9, phi=0.3, scale=1.0) -> Workload:
    """One (2,2,0) voice whose frequency is exactly linear in time:
    F_phi = (f0 + fdot t)/2 (so F_V = m F_phi = f0 + fdot t), F_r = 0, phase
    the exact quadratic integral, constant amplitude; on a uniform grid of
    Nf bins spanning the swept band with margins on both sides."""
    t = np.linspace(0.0, T, K)
    Fphi = 0.5 * (f0 + fdot * t)
    Phiphi = 0.5 * (Phi0 + 2 * math.pi * (f0 * t + 0.5 * fdot * t * t))
    traj = Trajectory(t=t, Fphi=Fphi, Fr=np.zeros(K), Phiphi=Phiphi, Phir=np.zeros(K),
                      p=np.full(K, 10.0), e=np.zeros(K))
    fa, fb = sorted([f0, f0 + fdot * T])
    span = fb - fa
    f = np.linspace(fa - 0.05 * span, fb + 0.05 * span, Nf)
    f = f[f > 0]
    return Workload(traj=traj, l=np.array([2], np.int32), m=np.array([2], np.int32),
                    n=np.array([0], np.int32), A=np.full((1, K), A0, np.complex128),
                    theta=theta, phi=phi, scale=scale, f=f, meta=dict(name="linear_chirp"))

"""Toy inspiral trajectory (oracle, test infrastructure).

Sec. 2.1: the adiabatic orbit is integrated to a sparse set of knots before
the mode sum.  The toy orbit-averaged fluxes of the synthetic workloads
(Peters-type, in the semi-latus rectum p and eccentricity e):

    dp/dt = -(64/5) q (1-e^2)^{3/2} p^-3 (1 + 7 e^2/8) / M_s
    de/dt = -(304/15) q e (1-e^2)^{3/2} p^-4 (1 + 121 e^2/304) / M_s
    dPhi_phi/dt = Omega_phi / M_s,   dPhi_r/dt = Omega_r / M_s
    Omega_phi = p^{-3/2} (1-e^2)^{3/2},   Omega_r = Omega_phi sqrt(1 - 6/p)

q = mu/M, M_s = M G M_sun / c^3; from t = 0 to T or to the plunge
p = 6 + 2e + 0.1; K knots uniform in [0, t_end].  Integrated with SciPy's
DOP853 at a tighter tolerance than the device integrator, the knots read
from its dense output.

Closed forms that pin it (tests): for e = 0, with a = (256/5) q / M_s,
p^4 = p0^4 - a t, Phi_phi = 8 (p0^{5/2} - p^{5/2}) / (5 a M_s) and the plunge at
t = (p0^4 - 6.1^4) / a; along any orbit p e^{-12/19} (1 + 121 e^2/304)^{-870/2299}
is constant (d ln p / d ln e of the two fluxes integrates to it).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp

G_MSUN_OVER_C3 = 4.925490947641267e-6  # s


def rhs(q, Ms):
    def f(_t, y):
        p, e = y[0], y[1]
        w = (1.0 - e * e) ** 1.5
        om_phi = p ** -1.5 * w
        return [-(64.0 / 5.0) * q * w * p ** -3 * (1.0 + 7.0 * e * e / 8.0) / Ms,
                -(304.0 / 15.0) * q * e * w * p ** -4 * (1.0 + 121.0 * e * e / 304.0) / Ms,
                om_phi / Ms,
                om_phi * math.sqrt(1.0 - 6.0 / p) / Ms]
    return f


def trajectory(M, mu, p0, e0, T, K, Phiphi0=0.0, Phir0=0.0):
    """Rows t, F_phi, F_r, Phi_phi, Phi_r, p, e at the K knots ([7, K])."""
    Ms = M * G_MSUN_OVER_C3
    q = mu / M

    def plunge(_t, y):
        return y[0] - (6.0 + 2.0 * y[1] + 0.1)
    plunge.terminal = True
    plunge.direction = -1
    sol = solve_ivp(rhs(q, Ms), (0.0, T), [p0, e0, Phiphi0, Phir0], method="DOP853", rtol=1e-13,
                    atol=[1e-13, 1e-15, 1e-10, 1e-10], dense_output=True, events=plunge)
    t_end = float(sol.t_events[0][0]) if sol.t_events[0].size else float(T)
    t = np.linspace(0.0, t_end, K)
    y = sol.sol(t)
    p, e = y[0], y[1]
    om_phi = p ** -1.5 * (1.0 - e * e) ** 1.5
    om_r = om_phi * np.sqrt(1.0 - 6.0 / p)
    two_pi_Ms = 2.0 * math.pi * Ms
    return np.vstack([t, om_phi / two_pi_Ms, om_r / two_pi_Ms, y[2], y[3], p, e])


def peters_invariant(p, e):
    """p e^{-12/19} (1 + 121 e^2/304)^{-870/2299}: constant along the flow."""
    return p * e ** (-12.0 / 19.0) * (1.0 + 121.0 * e * e / 304.0) ** (-870.0 / 2299.0)

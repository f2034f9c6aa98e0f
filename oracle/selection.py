"""Mode selection by power (oracle, test infrastructure).

Sec. 2.1: the waveform keeps the modes whose share of the total power is
above a threshold.  The share is taken at every knot of the trajectory and a
mode is kept if it passes at one knot at least (the union over knots):

    keep mu  <=>  exists i:  |A_mu(t_i)|^2 > eps * sum_nu |A_nu(t_i)|^2,

with |A|^2 = re^2 + im^2 (each square rounded, then the sum).
"""
from __future__ import annotations

import numpy as np


def select_modes(A, eps):
    """Indices (table order) of the rows of A [Nm, K] (complex amplitude knot
    values) kept at threshold eps."""
    A = np.asarray(A, np.complex128)
    if A.shape[0] == 0:
        return np.zeros(0, np.int64)
    pw = A.real * A.real + A.imag * A.imag
    total = pw.sum(axis=0)
    keep = np.any(pw > eps * total[None, :], axis=1)
    return np.nonzero(keep)[0]


def margin(A, eps):
    """Per row, the largest ratio |A_mu(t_i)|^2 / (eps * total_i) over knots:
    rows with a ratio within rounding of 1 are decided by the summation order."""
    A = np.asarray(A, np.complex128)
    pw = A.real * A.real + A.imag * A.imag
    total = pw.sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.max(pw / (eps * total[None, :]), axis=1)

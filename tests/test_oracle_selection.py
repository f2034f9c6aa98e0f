"""Pins of the oracle's mode selection (Sec. 2.1, power share at every knot,
union over knots) by brute force on small tables and by the closed form of a
table whose time dependence is common to all modes."""
import numpy as np

import workloads as W
from oracle.selection import select_modes


def brute(A, eps):
    Nm, K = A.shape
    out = []
    for mu in range(Nm):
        for i in range(K):
            tot = sum(abs(A[nu, i]) ** 2 for nu in range(Nm))
            if abs(A[mu, i]) ** 2 > eps * tot * (1 + 1e-12):
                out.append(mu)
                break
    return out


def test_union_over_knots_and_strict_threshold():
    # row 0 dominates everywhere; row 1 passes only at knot 2; row 2 never;
    # row 3 sits exactly on the threshold at knot 0 (kept only if strictly above)
    A = np.array([[1.0, 1.0, 1.0, 1.0],
                  [1e-4, 1e-4, 0.9, 1e-4],
                  [1e-5, 1e-5, 1e-5, 1e-5],
                  [0.0, 0.0, 0.0, 0.0]], np.complex128)
    eps = 0.05
    kept = list(select_modes(A, eps))
    assert kept == [0, 1]
    # exactly at the threshold: a row with power eps * total is not kept
    B = np.array([[3.0, 3.0], [1.0, 1.0]], np.complex128)  # powers 9 and 1, total 10
    assert list(select_modes(B, 0.1)) == [0]
    assert list(select_modes(B, 0.0999)) == [0, 1]


def test_brute_force_random_tables():
    rng = np.random.default_rng(2)
    for trial in range(20):
        Nm, K = rng.integers(1, 9), rng.integers(1, 6)
        A = (rng.lognormal(0, 2, (Nm, K)) * np.exp(1j * rng.uniform(0, 6.3, (Nm, K))))
        eps = 10 ** rng.uniform(-4, -0.5)
        got = list(select_modes(A, eps))
        ref = brute(A, eps)
        # rows within 1e-12 of the threshold may go either way
        amb = [mu for mu in range(Nm) if (mu in got) != (mu in ref)]
        for mu in amb:
            r = max(abs(A[mu, i]) ** 2 / (eps * sum(abs(A[nu, i]) ** 2 for nu in range(Nm))) for i in range(K))
            assert abs(r - 1) < 1e-9, (trial, mu, r)


def test_common_time_factor_reduces_to_time_independent_rule():
    # A = a(mu) g(t) with real positive g: the share is |a|^2 / sum |a|^2 at
    # every knot, the rule the synthetic 3842-mode workload applies on the host
    full = W.inspiral_3842_modes(eps=0.0)
    sel = W.inspiral_3842_modes()
    kept = select_modes(full.A, 1e-5)
    assert kept.size == sel.l.size == 3842
    np.testing.assert_array_equal(full.l[kept], sel.l)
    np.testing.assert_array_equal(full.n[kept], sel.n)

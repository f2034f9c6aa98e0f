"""Polynomial coefficients of the device sin/cos kernels (csrc/evalcore.hpp).

On r in [-pi/4, pi/4], with z = r^2:
    sin r = r + r z P(z),          P of degree 5 (FP64 path), 2 (FP32, mixed path),
    cos r = 1 - z/2 + z^2 Q(z),    Q of degree 5 (FP64 path), 2 (FP32, mixed path),
with P, Q the least-squares fits (in 60-digit arithmetic) of
(sin sqrt(z) - sqrt(z)) / z^(3/2) and (cos sqrt(z) - 1 + z/2) / z^2 on 400
Chebyshev nodes of [0, (pi/4)^2].  Also prints the two-part split of pi/2
used by the range reduction (33-bit head, rounded remainder) and the maximum
approximation errors (relative for sin, absolute for cos).

    python -m paper_2307_12585_amd.gen_sincos_coeffs
"""
from __future__ import annotations

import mpmath as mp


def fit(fun, deg, z_max, npts=400):
    nodes = [z_max * (1 - mp.cos(mp.pi * (k + mp.mpf(1) / 2) / npts)) / 2 for k in range(npts)]
    A = mp.matrix(npts, deg + 1)
    b = mp.matrix(npts, 1)
    for i, z in enumerate(nodes):
        for j in range(deg + 1):
            A[i, j] = z ** j
        b[i] = fun(z)
    x = mp.lu_solve(A.T * A, A.T * b)
    return [x[j] for j in range(deg + 1)]


def main():
    mp.mp.dps = 60
    R = mp.pi / 4
    Z = R * R

    def p_sin(z):
        if z == 0:
            return mp.mpf(-1) / 6
        r = mp.sqrt(z)
        return (mp.sin(r) - r) / r ** 3

    def p_cos(z):
        if z == 0:
            return mp.mpf(1) / 24
        return (mp.cos(mp.sqrt(z)) - 1 + z / 2) / (z * z)

    grid = [R * k / 400 for k in range(401)]
    for deg, what in ((5, "FP64"), (2, "FP32")):
        ps = fit(p_sin, deg, Z)
        pc = fit(p_cos, deg, Z)
        es = max(abs(mp.sin(r) - (r + r ** 3 * sum(ps[j] * (r * r) ** j for j in range(deg + 1)))) / abs(mp.sin(r))
                 for r in grid[1:])
        ec = max(abs(mp.cos(r) - (1 - r * r / 2 + (r * r) ** 2 * sum(pc[j] * (r * r) ** j for j in range(deg + 1))))
                 for r in grid)
        print(f"{what} sin P (ascending):", [repr(float(c)) for c in ps])
        print(f"{what} cos Q (ascending):", [repr(float(c)) for c in pc])
        print(f"{what} approximation error: sin {float(es):.2e} (relative), cos {float(ec):.2e}")
    head = mp.mpf(1.5707963267341256)  # pi/2 to 33 bits
    print("pi/2 split:", repr(float(head)), repr(float(mp.pi / 2 - head)))


if __name__ == "__main__":
    main()

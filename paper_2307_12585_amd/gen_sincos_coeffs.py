"""Polynomial coefficients of the device sin/cos kernels (csrc/evalcore.hpp).

With z = r^2:
    sin r = r + r z P(z),   cos r = 1 - z/2 + z^2 Q(z),
with P, Q the least-squares fits (in 60-digit arithmetic) of
(sin sqrt(z) - sqrt(z)) / z^(3/2) and (cos sqrt(z) - 1 + z/2) / z^2 on 400
Chebyshev nodes of [0, R^2]:
    FP64 path: R = pi/2 (the argument reduced by pi), P, Q of degree 7;
    FP32 (mixed) path: R = pi/4 (reduced by pi/2), P, Q of degree 2.
Also prints the two-part splits of pi and pi/2 used by the range reductions
(head to 34 and 33 bits, so that k times it is exact for the multiples that
occur; rounded remainder) and the maximum approximation errors (relative
for sin, absolute for cos).

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


def coefficients():
    """{path: (P, Q, sin error, cos error)} for the two device kernels."""
    mp.mp.dps = 60

    def p_sin(z):
        if z == 0:
            return mp.mpf(-1) / 6
        r = mp.sqrt(z)
        return (mp.sin(r) - r) / r ** 3

    def p_cos(z):
        if z == 0:
            return mp.mpf(1) / 24
        return (mp.cos(mp.sqrt(z)) - 1 + z / 2) / (z * z)

    out = {}
    for what, R, deg in (("FP64", mp.pi / 2, 7), ("FP32", mp.pi / 4, 2)):
        Z = R * R
        grid = [R * k / 400 for k in range(401)]
        ps = fit(p_sin, deg, Z)
        pc = fit(p_cos, deg, Z)
        es = max(abs(mp.sin(r) - (r + r ** 3 * sum(ps[j] * (r * r) ** j for j in range(deg + 1)))) / abs(mp.sin(r))
                 for r in grid[1:])
        ec = max(abs(mp.cos(r) - (1 - r * r / 2 + (r * r) ** 2 * sum(pc[j] * (r * r) ** j for j in range(deg + 1))))
                 for r in grid)
        out[what] = ([float(c) for c in ps], [float(c) for c in pc], float(es), float(ec))
    return out


def splits():
    """(head, remainder) of pi and of pi/2."""
    mp.mp.dps = 60
    h2 = mp.mpf(1.5707963267341256)  # pi/2 to 33 bits
    return {"pi": (float(2 * h2), float(mp.pi - 2 * h2)), "pi/2": (float(h2), float(mp.pi / 2 - h2))}


def main():
    for what, (ps, pc, es, ec) in coefficients().items():
        print(f"{what} sin P (ascending):", [repr(c) for c in ps])
        print(f"{what} cos Q (ascending):", [repr(c) for c in pc])
        print(f"{what} approximation error: sin {es:.2e} (relative), cos {ec:.2e}")
    for name, (h, l) in splits().items():
        print(f"{name} split:", repr(h), repr(l))


if __name__ == "__main__":
    main()

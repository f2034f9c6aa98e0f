"""The sin/cos constants of the device code (csrc/evalcore.hpp) are those the
committed generator produces (paper_2307_12585_amd/gen_sincos_coeffs.py:
least-squares fits in 60-digit arithmetic), and the FP64 kernel's arithmetic,
replayed on the host in IEEE double with fused multiply-adds, is accurate to
a few units in the last place over the phases that occur."""
import math
import os
import re

import numpy as np

from paper_2307_12585_amd import gen_sincos_coeffs as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "paper_2307_12585_amd", "csrc", "evalcore.hpp")).read()


def body(name):
    i = SRC.index(f"void {name}(")
    return SRC[i:SRC.index("\n}\n", i)]


def literals(text):
    return [float(x) for x in re.findall(r"-?\d+\.\d+(?:e[-+]?\d+)?", text)]


def test_fp64_constants_are_the_generators():
    ps, pc, es, ec = G.coefficients()["FP64"]
    b = body("sincos_cw")
    lit = literals(b)
    head, rem = G.splits()["pi"]
    assert head in lit and rem in lit and float(repr(1 / math.pi)) in lit
    for c in ps + pc:
        assert c in lit, c
    assert es < 1e-17 and ec < 1e-18


def test_fp32_constants_are_the_generators():
    ps, pc, _, _ = G.coefficients()["FP32"]
    lit = literals(body("sincos_mixed"))
    head, rem = G.splits()["pi/2"]
    assert head in lit and rem in lit
    for c in ps + pc:
        assert float(np.float32(c)) in [float(np.float32(x)) for x in lit], c


def fma(a, b, c):
    """a b + c rounded once (exact product and sum in Python integers' rationals)."""
    from fractions import Fraction
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def device_sincos(x, ps, pc, head, rem):
    k = float(np.rint(x * float(repr(1 / math.pi))))
    r = fma(-k, head, x)
    r = fma(-k, rem, r)
    z = r * r
    s = ps[-1]
    for c in reversed(ps[:-1]):
        s = fma(s, z, c)
    s_r = fma(r * z, s, r)
    c = pc[-1]
    for q in reversed(pc[:-1]):
        c = fma(c, z, q)
    c_r = fma(z * z, c, fma(-0.5, z, 1.0))
    sg = -1.0 if int(k) & 1 else 1.0
    return sg * s_r, sg * c_r


def test_fp64_kernel_accuracy_over_the_phases_that_occur():
    import mpmath as mp
    mp.mp.dps = 40
    ps, pc, _, _ = G.coefficients()["FP64"]
    head, rem = G.splits()["pi"]
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(-4000, 4000, 300), rng.uniform(-4, 4, 100),
                         np.array([0.0, math.pi / 2, -math.pi / 2, math.pi, 1e-9])])
    worst = 0.0
    for x in xs:
        s, c = device_sincos(float(x), ps, pc, head, rem)
        worst = max(worst, abs(s - float(mp.sin(mp.mpf(float(x))))), abs(c - float(mp.cos(mp.mpf(float(x))))))
    # two units in the last place of a result of size 1 (measured 1.9e-16)
    assert worst <= 4.5e-16, worst

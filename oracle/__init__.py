"""CPU oracle for the frequency-domain EMRI mode sum (test infrastructure).

A plain, slow, FP64 NumPy/SciPy implementation of what the hot path
computes, written from the paper's method (Sec. 2.2, Eqs. cubic_equation,
SPAintegral2, extendedspa1) in its own order and notation:

  splines of the trajectory and amplitudes (Sec. 2.1)  -> explicit voices
  (Eq. wave_voice) -> all roots of F_V(t) = +-f (Eq. cubic_equation) ->
  per-root third-order SPA factor (Eq. extendedspa1) -> sum over voices ->
  plus/cross polarizations (Eq. main_wave).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library and must never
be used as a fallback for it.

Precision: FP64 throughout except the large phase 2 pi f t - Phi(t), which is
formed in x87 extended precision (numpy.longdouble) before reduction.
"""
from .harmonics import swsh, swsh_dtheta
from .special import W, G, G_airy, G_bessel
from .waveform import (Voice, splines, voices_from_modes, voice_pieces, waveform,
                       waveform_voices)
from .likelihood import inner_product, whittle_loglike

__all__ = [
    "swsh", "swsh_dtheta", "W", "G", "G_airy", "G_bessel", "Voice", "splines",
    "voices_from_modes", "voice_pieces", "waveform", "waveform_voices",
    "inner_product", "whittle_loglike",
]

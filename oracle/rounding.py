"""Rounding of real numbers to the narrow floating-point formats that the
low-precision sketch variants feed to the matrix cores.

The paper fixes no arithmetic precision for the sketch (Alg. 1 step 2); the
low-precision variants are defined as: round every entry of Pi and of the
data to the format (round to nearest, ties to even), then form the exact
product. These functions are that rounding, written from the format
definitions:

* bfloat16: 1 sign bit, 8 exponent bits (bias 127, the FP32 range, with
  subnormals down to 2^-133), 7 stored significand bits (8 significant bits).

Input and output are FP64 arrays; the results are exactly representable in
the format.
"""

import numpy as np

BF16_SIG_BITS = 8                     # significant bits, implicit one included
BF16_EMIN = -126                      # exponent of the smallest normal number
BF16_MAX = (2.0 - 2.0 ** -7) * 2.0 ** 127


def _round_sig(x, sig_bits, emin, max_finite, overflow_to_inf=True):
    """Round x to nearest (ties to even) in a binary format with `sig_bits`
    significant bits, smallest normal exponent `emin` (gradual underflow
    below it) and largest finite value `max_finite`."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    fin = np.isfinite(x) & (x != 0)
    ax = np.abs(x[fin])
    # exponent e with 2^e <= |x| < 2^(e+1), clamped at emin (subnormal range)
    _, e = np.frexp(ax)                  # ax = f * 2^e, 0.5 <= f < 1
    e = np.maximum(e - 1, emin)
    ulp = np.ldexp(1.0, e - (sig_bits - 1))
    r = np.rint(ax / ulp) * ulp          # np.rint rounds half to even; ax / ulp is exact
    if overflow_to_inf:
        # the rounding boundary above max_finite is max_finite + ulp(max_finite) / 2
        half = np.ldexp(1.0, int(np.floor(np.log2(max_finite))) - sig_bits)
        r = np.where(ax >= max_finite + half, np.inf, np.minimum(r, max_finite))
    out[fin] = np.copysign(r, x[fin])
    out[~np.isfinite(x)] = x[~np.isfinite(x)]
    return out


def round_bf16(x):
    """x rounded to the nearest bfloat16 (ties to even); overflow gives inf."""
    return _round_sig(x, BF16_SIG_BITS, BF16_EMIN, BF16_MAX)

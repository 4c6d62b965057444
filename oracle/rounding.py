"""Rounding of real numbers to the narrow floating-point formats that the
low-precision sketch variants feed to the matrix cores.

The paper fixes no arithmetic precision for the sketch (Alg. 1 step 2); the
low-precision variants are defined as: round every entry of Pi and of the
data to the format (round to nearest, ties to even), then form the exact
product. These functions are that rounding, written from the format
definitions:

* bfloat16: 1 sign bit, 8 exponent bits (bias 127, the FP32 range, with
  subnormals down to 2^-133), 7 stored significand bits (8 significant bits).
* FP8 E4M3 (the OCP 8-bit format "E4M3FN"): 1 sign bit, 4 exponent bits
  (bias 7), 3 stored significand bits; largest finite value 448, smallest
  normal 2^-6, subnormal spacing 2^-9; no infinities.
* E8M0 block scales (the OCP microscaling shared-exponent format): a power of
  two 2^e, e in [-127, 127].

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


E4M3_SIG_BITS = 4
E4M3_EMIN = -6
E4M3_MAX = 448.0
MX_BLOCK = 32                         # rows sharing one data scale


def round_bf16(x):
    """x rounded to the nearest bfloat16 (ties to even); overflow gives inf."""
    return _round_sig(x, BF16_SIG_BITS, BF16_EMIN, BF16_MAX)


def round_e4m3(x):
    """x rounded to the nearest FP8 E4M3 value (ties to even). Magnitudes at or
    beyond the rounding boundary above 448 saturate to +-448 (the callers
    scale their data so that this never happens)."""
    r = _round_sig(x, E4M3_SIG_BITS, E4M3_EMIN, E4M3_MAX, overflow_to_inf=False)
    return np.clip(r, -E4M3_MAX, E4M3_MAX)


def mx_scale_exponent(amax):
    """Exponent e of the data scale 2^e of a block whose largest magnitude is
    amax: the smallest integer with amax <= 448 * 2^e (so the scaled block
    fits the E4M3 range without saturating), clamped to the E8M0 range
    [-127, 127]; e = 0 for an all-zero block."""
    amax = np.asarray(amax, dtype=np.float64)
    e = np.zeros(amax.shape, dtype=np.int64)
    pos = amax > 0
    m, ex = np.frexp(amax[pos] / E4M3_MAX)     # amax / 448 = m 2^ex, 0.5 <= m < 1
    e[pos] = np.where(m == 0.5, ex - 1, ex)    # exact powers of two need no extra step
    return np.clip(e, -127, 127)


def quantize_e4m3_blocks(X, row0=0):
    """The E4M3 data operand with E8M0 block scales, dequantized: for each
    column and each block of MX_BLOCK consecutive global rows (rows
    [32 b, 32 b + 32) of the whole matrix; X holds rows row0 .. row0 +
    len(X) - 1 and row0 is a multiple of 32), scale 2^e with e =
    mx_scale_exponent(max |x| over the block), value round_e4m3(x 2^-e) 2^e."""
    X = np.asarray(X, dtype=np.float64)
    assert row0 % MX_BLOCK == 0
    out = np.empty_like(X)
    for b0 in range(0, X.shape[0], MX_BLOCK):
        blk = X[b0:b0 + MX_BLOCK]
        e = mx_scale_exponent(np.max(np.abs(blk), axis=0))
        sc = np.ldexp(1.0, e)
        out[b0:b0 + MX_BLOCK] = round_e4m3(blk / sc) * sc
    return out

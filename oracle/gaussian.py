"""Standard normal variates from pairs of 32-bit words, by the Box-Muller
transform (G. E. P. Box, M. E. Muller, "A note on the generation of random
normal deviates", Ann. Math. Stat. 29, 1958).

The paper only fixes the distribution: Pi(i, j) ~ N(0, 1/k), i.i.d. (Alg. 1
step 2). The transform used on both sides of the parity check:

  u   = ((a >> 8) + 1) * 2^-24          in (0, 1]   (never 0, so log u is finite)
  phi = (b >> 8) * 2^-24                in [0, 1)   (a fraction of a full turn)
  rad = sqrt(-2 ln u)
  z_cos = rad * cos(2 pi phi),  z_sin = rad * sin(2 pi phi)

Both uniforms are 24-bit dyadic rationals, exact in FP32 and FP64, so the two
sides differ only in the rounding of log, sqrt, cos and sin.

A Philox call gives words (w0, w1, w2, w3); sketch row c uses
  c mod 4 == 0 -> z_cos(w0, w1),  1 -> z_sin(w0, w1),
  c mod 4 == 2 -> z_cos(w2, w3),  3 -> z_sin(w2, w3).

Parity: pinned by distribution tests (moments, Kolmogorov-Smirnov) and by the
closed-form variance of the JL inner-product estimator (tests/test_oracle_rng.py).
"""

import numpy as np

_TWO_M24 = 2.0 ** -24


def uniforms(a, b):
    """The two 24-bit uniforms (u in (0,1], phi in [0,1)) of the transform."""
    a = np.asarray(a, dtype=np.uint32)
    b = np.asarray(b, dtype=np.uint32)
    u = ((a >> np.uint32(8)).astype(np.float64) + 1.0) * _TWO_M24
    phi = (b >> np.uint32(8)).astype(np.float64) * _TWO_M24
    return u, phi


def box_muller(a, b):
    """Return (z_cos, z_sin), two independent N(0, 1) variates in FP64."""
    u, phi = uniforms(a, b)
    rad = np.sqrt(-2.0 * np.log(u))
    ang = 2.0 * np.pi * phi
    return rad * np.cos(ang), rad * np.sin(ang)


def normals_from_words(w0, w1, w2, w3):
    """The four N(0,1) variates of one Philox call, in lane order 0..3."""
    z0, z1 = box_muller(w0, w1)
    z2, z3 = box_muller(w2, w3)
    return z0, z1, z2, z3

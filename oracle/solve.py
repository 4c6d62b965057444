"""SMP-PCA end to end (Alg. 1): one pass, sampling, rescaled-JL estimates,
WAltMin. Parameters follow the paper: rank r, samples m, sketch size k,
iterations T (Section 2.1), plus the seed of the counter-based generator.
"""

import math

import numpy as np

from . import sketch as _sketch
from . import sample as _sample
from . import multinomial as _multinomial
from . import srht as _srht
from . import estimate as _estimate
from . import waltmin as _waltmin


def default_m(n1, n2, r):
    """m = 4 n r log n with n = max(n1, n2) and the natural log (Section 4,
    "Sample complexity"; n for unequal sizes per Section 3)."""
    n = max(n1, n2)
    return 4.0 * n * r * math.log(n)


def smp_pca(A, B, r, k, m, T, seed, split=False, sketch_fmt=None, sampler="binomial", sketch_kind="gaussian"):
    """Run Alg. 1. A: d x n1, B: d x n2 or None (A = B, Section 3 Remark 3).
    sketch_fmt: None for the FP64 pass, or a narrow format ("bf16", "fp8") whose
    rounded operands form the sketches (``oracle.sketch.sketch_lowp``).
    sampler: "binomial" (Alg. 1 step 3, ``oracle.sample``) or "multinomial"
    (the row-wise sampler of Appendix D, ``oracle.multinomial``).
    sketch_kind: "gaussian" (Alg. 1 step 2) or "srht" (the subsampled
    randomized Hadamard transform of the Spark implementation, ``oracle.srht``;
    FP64 only).
    Returns a dict with the output factors and every intermediate:
      At, Bt, na2, nb2      sketches and squared column norms (step 2)
      omega                  oracle.sample.Omega (step 3)
      mt                     M~ on omega (step 4)
      U, V                   WAltMin output (step 5), U V^T the approximation
      Uc, sigma, Vc          canonical SVD form of U V^T
    """
    if sketch_kind == "srht":
        assert sketch_fmt is None, "the SRHT sketch is defined in FP64 only"
        At, Bt, na2, nb2 = _srht.sketch(A, B, seed, k)
    elif sketch_fmt is None:
        At, Bt, na2, nb2 = _sketch.sketch(A, B, seed, k)
    else:
        At, Bt, na2, nb2 = _sketch.sketch_lowp(A, B, seed, k, sketch_fmt)
    if sampler == "multinomial":
        om = _multinomial.sample(na2, nb2, m, seed, T=T, split=split)
    elif sampler == "binomial":
        om = _sample.sample(na2, nb2, m, seed, T=T, split=split)
    else:
        raise ValueError(f"unknown sampler {sampler!r}")
    mt = _estimate.estimate(At, Bt, na2, nb2, om.rows, om.cols)
    res = _waltmin.waltmin(om.n1, om.n2, om.rows, om.cols, om.w, mt, r, T, na2, om.FA,
                           subset=om.subset)
    Uc, s, Vc = _waltmin.canonical(res["U"], res["V"])
    return dict(At=At, Bt=Bt, na2=na2, nb2=nb2, omega=om, mt=mt,
                U=res["U"], V=res["V"], U0=res["U0"], S0=res["S0"], V0=res["V0"],
                trimmed=res["trimmed"], Uc=Uc, sigma=s, Vc=Vc)

"""The two comparison methods of the paper (Section 1 footnote, Section 4),
as plain FP64 definitions. Test infrastructure, like the rest of this package.

* SVD(A~^T B~): sketch A and B with the same Pi as Alg. 1 step 2 and take the
  top-r SVD of the product of the sketches, without the rescaling of Eq. (2)
  (the "straightforward idea" of the Section 1 footnote; Figures 2(b), 4(b)).
* LELA: the two-pass method the paper compares against (Section 4, "Comparison
  of SMP-PCA and LELA"; Remark 1 of Section 3): the first pass computes the
  column norms, the second pass the exact entries (A^T B)_ij on the sample
  drawn from Eq. (1); WAltMin (Alg. 2) then runs on those exact entries. It is
  SMP-PCA with M~_ij replaced by A_i^T B_j.
"""

import numpy as np

from . import evaluate, multinomial, sample, waltmin
from .sketch import sketch


def svd_of_sketches(At, Bt, r):
    """Top-r SVD of At^T Bt (At: k x n1, Bt: k x n2): (U, sigma, V) with
    orthonormal U, V and U diag(sigma) V^T the best rank-r approximation."""
    X = np.asarray(At, dtype=np.float64).T @ np.asarray(Bt, dtype=np.float64)
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    return U[:, :r], s[:r], Vt[:r].T


def svd_of_sketch_product(A, B, r, k, seed):
    """SVD(A~^T B~) with the Gaussian Pi of Alg. 1 step 2 (same counter spec)."""
    At, Bt, _, _ = sketch(A, B, seed, k)
    return svd_of_sketches(At, Bt, r)


def column_norms2(A):
    """||A_i||^2 of every column, FP64 (LELA's first pass)."""
    A = np.asarray(A)
    out = np.zeros(A.shape[1])
    for l0 in range(0, A.shape[0], 16384):
        a = np.asarray(A[l0:l0 + 16384], dtype=np.float64)
        out += np.einsum("li,li->i", a, a)
    return out


def lela(A, B, r, m, T, seed, split=False, sampler="binomial"):
    """LELA: exact norms, the sample of Eq. (1) (the same coins as Alg. 1 step
    3, or Appendix D's row-wise draws), exact entries on it, WAltMin, and the
    canonical form. Returns dict(Uc, sigma, Vc, omega, mt)."""
    na2 = column_norms2(A)
    nb2 = column_norms2(B)
    if sampler == "multinomial":
        om = multinomial.sample(na2, nb2, m, seed, T=T, split=split)
    else:
        om = sample.sample(na2, nb2, m, seed, T=T, split=split)
    M = evaluate.product(A, B)                    # the second pass: exact A^T B, then the sampled entries
    mt = M[om.rows, om.cols]
    res = waltmin.waltmin(om.n1, om.n2, om.rows, om.cols, om.w, mt, r, T, na2, om.FA, subset=om.subset)
    Uc, s, Vc = waltmin.canonical(res["U"], res["V"])
    return dict(Uc=Uc, sigma=s, Vc=Vc, omega=om, mt=mt, na2=na2, nb2=nb2)

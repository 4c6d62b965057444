"""Rescaled-JL estimates on Omega (Eq. (2); Alg. 1 step 4).

  M~(i, j) = ||A_i|| * ||B_j|| * <A~_i, B~_j> / (||A~_i|| * ||B~_j||)

computed only for (i, j) in Omega (the paper never forms M~). Equivalently
M~ = D_A A~^T B~ D_B with (D_A)_ii = ||A_i|| / ||A~_i||, (D_B)_jj = ||B_j|| / ||B~_j||
(Appendix B, the compact form stated before Lemma B.4).

Readings where the paper is silent: the cosine is clamped to [-1, 1] (it can
leave that interval only by rounding), and M~(i, j) = 0 if any of the four
norms is 0.
"""

import numpy as np


def sketch_column_norms(St):
    """||A~_i|| for every column of a k x n sketch, FP64."""
    St = np.asarray(St, dtype=np.float64)
    return np.sqrt((St * St).sum(axis=0))


def estimate(At, Bt, na2, nb2, rows, cols, chunk=65536):
    """M~ on the listed entries. At: k x n1, Bt: k x n2 sketches; na2, nb2:
    squared column norms of A and B; rows, cols: entry coordinates."""
    At = np.asarray(At, dtype=np.float64)
    Bt = np.asarray(Bt, dtype=np.float64)
    sa = sketch_column_norms(At)
    sb = sketch_column_norms(Bt)
    na = np.sqrt(np.asarray(na2, dtype=np.float64))
    nb = np.sqrt(np.asarray(nb2, dtype=np.float64))
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    out = np.zeros(rows.size)
    for e0 in range(0, rows.size, chunk):
        r = rows[e0:e0 + chunk]
        c = cols[e0:e0 + chunk]
        dots = np.einsum("ke,ke->e", At[:, r], Bt[:, c])
        den = sa[r] * sb[c]
        ok = (den > 0) & (na[r] > 0) & (nb[c] > 0)
        cos = np.clip(np.where(ok, dots / np.where(ok, den, 1.0), 0.0), -1.0, 1.0)
        out[e0:e0 + chunk] = np.where(ok, na[r] * nb[c] * cos, 0.0)
    return out


def estimate_dense(At, Bt, na2, nb2):
    """The whole n1 x n2 matrix M~ by the compact form D_A A~^T B~ D_B (small
    problems and tests only; the method itself never forms it)."""
    At = np.asarray(At, dtype=np.float64)
    Bt = np.asarray(Bt, dtype=np.float64)
    sa = sketch_column_norms(At)
    sb = sketch_column_norms(Bt)
    da = np.where(sa > 0, np.sqrt(na2) / np.where(sa > 0, sa, 1.0), 0.0)
    db = np.where(sb > 0, np.sqrt(nb2) / np.where(sb > 0, sb, 1.0), 0.0)
    return (da[:, None] * (At.T @ Bt)) * db[None, :]

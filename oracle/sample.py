"""Biased entrywise sampling (Eq. (1); Alg. 1 step 3; Alg. 2 steps 2-3).

  q_ij   = m * ( ||A_i||^2 / (2 n2 ||A||_F^2) + ||B_j||^2 / (2 n1 ||B||_F^2) )   (Eq. (1))
  q^_ij  = min{1, q_ij}
  (i, j) is in Omega independently with probability q^_ij  (Alg. 1 step 3)
  w_ij   = 1 / q^_ij  (0 where q^_ij = 0)                  (Alg. 2 step 2)

Fixed evaluation order (so that both sides decide every coin identically from
the same squared norms):
  F_A    = sum_i ||A_i||^2, summed sequentially inside consecutive blocks of 256
           indices, then sequentially over the block sums;  F_B likewise
  den_A  = (2 * n2) * F_A;  den_B = (2 * n1) * F_B
  alpha_i = na2_i / den_A;  beta_j = nb2_j / den_B   (0 when the denominator is 0)
  q_ij   = m * (alpha_i + beta_j);  q^ = min(1, q)
  thr_ij = floor(q^_ij * 2^32)   (an integer in [0, 2^32])
  (i, j) in Omega  iff  x_ij < thr_ij,  x_ij = Philox(seed; TAG_SAMPLE) word for (i, j)
Every step is one IEEE-754 binary64 operation (no fused multiply-add).

Subsets for Alg. 2 step 3 (SPLIT mode): entry (i, j) goes to subset
  s_ij = floor(y_ij * (2T + 1) / 2^32),  y_ij = Philox(seed; TAG_SPLIT) word for (i, j),
which gives 2T+1 uniformly random subsets of equal expected size.

Omega is returned in row-major order (sorted by i, then j): a CSR listing.
"""

from dataclasses import dataclass

import numpy as np

from .philox import TAG_SAMPLE, TAG_SPLIT, stream_word_at

_TWO32 = 4294967296.0


def fixed_order_sum(x):
    """Sum of x (FP64): sequential within blocks of 256 in index order, then
    sequential over the block sums."""
    x = np.asarray(x, dtype=np.float64)
    if x.size == 0:
        return 0.0
    blocks = [np.cumsum(x[b:b + 256])[-1] for b in range(0, x.size, 256)]
    return float(np.cumsum(np.asarray(blocks, dtype=np.float64))[-1])


def marginals(na2, nb2):
    """alpha_i and beta_j of Eq. (1) (without the factor m), in the fixed order."""
    na2 = np.asarray(na2, dtype=np.float64)
    nb2 = np.asarray(nb2, dtype=np.float64)
    n1, n2 = na2.size, nb2.size
    FA, FB = fixed_order_sum(na2), fixed_order_sum(nb2)
    den_a = (2.0 * n2) * FA
    den_b = (2.0 * n1) * FB
    alpha = na2 / den_a if den_a > 0 else np.zeros(n1)
    beta = nb2 / den_b if den_b > 0 else np.zeros(n2)
    return alpha, beta, FA, FB


def probabilities(na2, nb2, m):
    """Dense q (n1 x n2) of Eq. (1); for small problems and tests."""
    alpha, beta, _, _ = marginals(na2, nb2)
    return float(m) * (alpha[:, None] + beta[None, :])


@dataclass
class Omega:
    n1: int
    n2: int
    rows: np.ndarray      # int64, row-major order
    cols: np.ndarray      # int64
    qhat: np.ndarray      # FP64, min(1, q) per sampled entry
    w: np.ndarray         # FP64, 1 / qhat
    subset: np.ndarray    # int64 subset id in [0, 2T], or None (REUSE mode)
    FA: float
    FB: float

    @property
    def nnz(self):
        return int(self.rows.size)

    def row_ptr(self):
        return np.concatenate([[0], np.cumsum(np.bincount(self.rows, minlength=self.n1))]).astype(np.int64)


def thresholds(alpha, beta, m):
    """q^ and the integer thresholds floor(q^ * 2^32) for a block of rows."""
    q = float(m) * (alpha[:, None] + beta[None, :])
    qhat = np.minimum(1.0, q)
    thr = np.floor(qhat * _TWO32).astype(np.uint64)
    return qhat, thr


def sample(na2, nb2, m, seed, T=None, split=False, row_chunk=256):
    """Draw Omega (Alg. 1 step 3). If split, also assign the 2T+1 subsets of
    Alg. 2 step 3."""
    alpha, beta, FA, FB = marginals(na2, nb2)
    n1, n2 = alpha.size, beta.size
    rows_l, cols_l, qh_l, sub_l = [], [], [], []
    jj = np.arange(n2, dtype=np.int64)
    for i0 in range(0, n1, row_chunk):
        i1 = min(n1, i0 + row_chunk)
        ii = np.arange(i0, i1, dtype=np.int64)
        qhat, thr = thresholds(alpha[i0:i1], beta, m)
        x = stream_word_at(seed, TAG_SAMPLE, ii[:, None], jj[None, :]).astype(np.uint64)
        take = x < thr
        r, c = np.nonzero(take)                       # row-major order
        rows_l.append(r + i0)
        cols_l.append(c)
        qh_l.append(qhat[r, c])
        if split:
            y = stream_word_at(seed, TAG_SPLIT, r + i0, c).astype(np.uint64)
            sub_l.append(((y * np.uint64(2 * T + 1)) >> np.uint64(32)).astype(np.int64))
    rows = np.concatenate(rows_l).astype(np.int64)
    cols = np.concatenate(cols_l).astype(np.int64)
    qh = np.concatenate(qh_l)
    w = np.where(qh > 0, 1.0 / np.where(qh > 0, qh, 1.0), 0.0)
    subset = np.concatenate(sub_l) if split else None
    return Omega(n1, n2, rows, cols, qh, w, subset, FA, FB)

"""Row-wise multinomial sampling of Omega (Appendix D, "Sampling").

Test infrastructure: the plain CPU definition that the GPU sampler is checked
against, bit for bit. Nothing in the product path imports it.

Appendix D replaces the n1 n2 independent coins of Alg. 1 step 3 by, for each
row i, a number of draws with replacement from the row's share of Eq. (1):

  m_i      = sum_j q_ij = m (||A_i||^2 / (2 ||A||_F^2) + 1 / (2 n1))
  q~_ij    = q_ij / m_i  (sums to 1 over j)

and locates each draw by binary search over the row's CDF, whose entries are
a linear function of the column index plus a prefix sum shared by all rows
(the paper's "linear shift and scale"), so a row costs O(m_i log n2).

Readings where Appendix D is silent or garbled (it writes ||A_i|| where the
row being sampled, ||A_1||, is meant, and n for both n1 and n2; the sizes
follow Eq. (1)):
  * m_i is real but a count is needed: c_i = floor(m_i) + [x_i < floor(frac(m_i) 2^32)]
    with x_i a Philox word (randomised rounding, E[c_i] = m_i);
  * draws with replacement; entry (i, j) drawn N_ij times is kept once with
    weight w_ij = N_ij / q_ij, so E[w_ij 1{(i,j) in Omega}] = 1, as 1/q^ is for
    the binomial coins (Alg. 2 step 2);
  * the CDF is integer so that both sides locate every draw identically:
    a_i = floor(alpha_i 2^52), b_j = floor(beta_j 2^52) with alpha, beta the
    fixed-order binary64 marginals of Eq. (1) (``oracle.sample.marginals``),
    CDF_i(j) = (j + 1) a_i + (b_0 + ... + b_j), total_i = CDF_i(n2 - 1) < 2^53;
    q_ij = m ((a_i + b_j) 2^-52), m_i = m (total_i 2^-52) (one rounding each).

Random streams (the Philox counter spec of ``oracle.philox``):
  TAG_ROWCOUNT = 5: x_i = word 0 of the call (col_block 0, row i);
  TAG_DRAW = 6: draw k of row i uses the call (col_block k // 2, row i); its
  64-bit uniform u is words (0, 1) for even k, (2, 3) for odd k, high word
  first; the draw's target is t = floor(u total_i / 2^64) in [0, total_i) and
  its column the smallest j with CDF_i(j) > t.
"""

import numpy as np

from .philox import TAG_SPLIT, stream_word_at, stream_words
from .sample import Omega, marginals

TAG_ROWCOUNT = 5
TAG_DRAW = 6

_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)
_TWO32 = 4294967296.0
SCALE_BITS = 52


def mulhi64(u, t):
    """floor(u * t / 2^64) for uint64 arrays u and t (t < 2^53), exact:
    schoolbook product of the 32-bit halves with explicit carries."""
    u = np.asarray(u, dtype=np.uint64)
    t = np.asarray(t, dtype=np.uint64)
    uh, ul = u >> _S32, u & _M32
    th, tl = t >> _S32, t & _M32
    p0 = ul * tl                       # < 2^64
    p1 = uh * tl                       # < 2^64
    p2 = ul * th                       # < 2^53 (th < 2^21)
    mid_lo = (p1 & _M32) + (p2 & _M32) + (p0 >> _S32)      # < 3 * 2^32
    mid_hi = (p1 >> _S32) + (p2 >> _S32) + (mid_lo >> _S32)
    return uh * th + mid_hi


def integer_weights(na2, nb2):
    """a (n1), b (n2) as uint64 fixed-point weights, the inclusive prefix sums
    of b, the row totals, and the marginals they come from."""
    alpha, beta, FA, FB = marginals(na2, nb2)
    scale = float(2 ** SCALE_BITS)
    a = np.floor(alpha * scale).astype(np.uint64)
    b = np.floor(beta * scale).astype(np.uint64)
    bcum = np.cumsum(b, dtype=np.uint64)
    n2 = b.size
    total = np.uint64(n2) * a + (bcum[-1] if n2 else np.uint64(0))
    return a, b, bcum, total, FA, FB


def row_counts(total, m, seed):
    """c_i: randomised rounding of m_i = m (total_i 2^-52)."""
    n1 = total.size
    mi = float(m) * (total.astype(np.float64) * 2.0 ** -SCALE_BITS)
    fl = np.floor(mi)
    thr = np.floor((mi - fl) * _TWO32).astype(np.uint64)
    x = stream_word_at(seed, TAG_ROWCOUNT, np.arange(n1, dtype=np.int64), np.zeros(n1, dtype=np.int64))
    return fl.astype(np.int64) + (x.astype(np.uint64) < thr).astype(np.int64), mi


def locate(t, a_row, bcum):
    """Smallest j with (j + 1) a_row + bcum[j] > t, elementwise (binary search
    over the integer CDF; t < the row total)."""
    n2 = bcum.size
    lo = np.zeros(t.shape, dtype=np.int64)
    hi = np.full(t.shape, n2 - 1, dtype=np.int64)
    while True:
        act = lo < hi
        if not act.any():
            return lo
        mid = (lo + hi) // 2
        cdf = (mid + 1).astype(np.uint64) * a_row + bcum[mid]
        right = cdf > t
        hi = np.where(act & right, mid, hi)
        lo = np.where(act & ~right, mid + 1, lo)


def draws(a, bcum, total, counts, seed):
    """Rows and columns of every draw, row by row in draw order."""
    n1 = a.size
    rows = np.repeat(np.arange(n1, dtype=np.int64), counts)
    first = np.concatenate([[0], np.cumsum(counts)[:-1]]) if n1 else np.zeros(0, dtype=np.int64)
    k = np.arange(rows.size, dtype=np.int64) - np.repeat(first, counts)
    w0, w1, w2, w3 = stream_words(seed, TAG_DRAW, rows, k // 2)
    odd = (k % 2) == 1
    hi_w = np.where(odd, w2, w0).astype(np.uint64)
    lo_w = np.where(odd, w3, w1).astype(np.uint64)
    u = (hi_w << _S32) | lo_w
    t = mulhi64(u, total[rows])
    cols = locate(t, a[rows], bcum)
    return rows, cols


def sample(na2, nb2, m, seed, T=None, split=False):
    """Omega by row-wise multinomial sampling (Appendix D), in row-major order,
    each entry once with its multiplicity folded into w. Same return type as
    ``oracle.sample.sample``; qhat holds q_ij (the expected number of draws,
    not clamped) and the extra attribute `count` holds N_ij."""
    a, b, bcum, total, FA, FB = integer_weights(na2, nb2)
    n1, n2 = a.size, b.size
    counts, _ = row_counts(total, m, seed)
    r, c = draws(a, bcum, total, counts, seed)
    keys, mult = np.unique(r * n2 + c, return_counts=True)     # sorted: row-major
    rows, cols = keys // n2, keys % n2
    q = float(m) * ((a[rows] + b[cols]).astype(np.float64) * 2.0 ** -SCALE_BITS)
    w = mult.astype(np.float64) / q
    subset = None
    if split:
        y = stream_word_at(seed, TAG_SPLIT, rows, cols).astype(np.uint64)
        subset = ((y * np.uint64(2 * T + 1)) >> np.uint64(32)).astype(np.int64)
    om = Omega(n1, n2, rows.astype(np.int64), cols.astype(np.int64), q, w, subset, FA, FB)
    om.count = mult.astype(np.int64)
    om.row_draws = counts
    return om

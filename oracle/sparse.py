"""The sketch of matrices given entry by entry, in any order (Section 1: the
entries of A and B may arrive in an arbitrary order, as in streaming logs;
Section 3, "Computation Complexity": step 1 costs O(nnz(A) k + nnz(B) k)).
Test infrastructure, like the rest of this package.

A matrix X (d x n) is given as COO triples (l, i, v): row l < d, column i < n,
value v. Every (l, i) occurs at most once (a repeated pair is an error: its
square would enter the column norm twice, so the norm would no longer be the
one of the matrix the entries describe; reading of the streaming model). The
sketch is the definition of Alg. 1 step 2 applied to the matrix the triples
describe,
    X~[:, i] = sum over the triples (l, i, v) of column i of  v Pi[:, l],
    ||X_i||^2 = sum over the same triples of v^2,
with Pi the Gaussian sketching matrix (``oracle.sketch``), its BF16 form
(Pi and the values rounded to bfloat16, the products exact; the norms of the
unrounded values, as in ``oracle.sketch.sketch_lowp``) or the SRHT
(``oracle.srht``). The order of the triples does not enter the definition.

Pi is formed only for the rows that occur (k values per distinct row), in
chunks of rows; each triple then adds v Pi[:, l] into its column.
"""

import numpy as np

from .gaussian import normals_from_words
from .philox import TAG_PI, stream_words
from . import srht as _srht


def check_entries(rows, cols, vals, d, n):
    """Validate one matrix's triples; returns them as (int64, int64, float64)
    arrays. Raises ValueError for an index out of range or a repeated pair."""
    rows = np.asarray(rows, dtype=np.int64).ravel()
    cols = np.asarray(cols, dtype=np.int64).ravel()
    vals = np.asarray(vals, dtype=np.float64).ravel()
    if not (rows.shape == cols.shape == vals.shape):
        raise ValueError("rows, cols and vals differ in length")
    if rows.size and (rows.min() < 0 or rows.max() >= d):
        raise ValueError("row index out of [0, d)")
    if cols.size and (cols.min() < 0 or cols.max() >= n):
        raise ValueError("column index out of [0, n)")
    key = cols * int(d) + rows
    if np.unique(key).size != key.size:
        raise ValueError("an entry (row, column) occurs more than once")
    return rows, cols, vals


def gaussian_columns(seed, k, l):
    """Z[:, l] (k x len(l)) of the Gaussian sketching matrix before its 1/sqrt(k),
    for an array of row indices l: lane (c mod 4) of the Box-Muller variates of
    the Philox call (c // 4, l) under the Pi tag."""
    l = np.asarray(l, dtype=np.int64)
    nb = (k + 3) // 4
    w = stream_words(seed, TAG_PI, l[:, None], np.arange(nb, dtype=np.int64)[None, :])
    z = np.stack(normals_from_words(*w), axis=-1).reshape(l.size, 4 * nb)[:, :k]
    return np.ascontiguousarray(z.T)


def pi_columns(seed, k, d, l, kind="gaussian", fmt=None):
    """Pi[:, l] for row indices l (k x len(l)), FP64. kind "gaussian" (fmt None
    or "bf16": Z rounded to bfloat16 before the 1/sqrt(k)) or "srht"."""
    if kind == "srht":
        if fmt is not None:
            raise ValueError("the SRHT is defined in full precision only")
        return _srht.pi_columns(seed, k, d, l)
    if kind != "gaussian":
        raise ValueError(f"unknown sketch {kind!r}")
    Z = gaussian_columns(seed, k, l)
    if fmt == "bf16":
        from .rounding import round_bf16
        Z = round_bf16(Z)
    elif fmt is not None:
        raise ValueError(f"unsupported format {fmt!r} for entry input")
    return Z / np.sqrt(float(k))


def sketch_entries(rows, cols, vals, d, n, seed, k, kind="gaussian", fmt=None, row_chunk=2048):
    """(Xt, nx2): the k x n sketch and the n squared column norms of the d x n
    matrix that the triples describe."""
    rows, cols, vals = check_entries(rows, cols, vals, d, n)
    Xt = np.zeros((k, n))
    nx2 = np.zeros(n)
    np.add.at(nx2, cols, vals * vals)
    v = vals
    if fmt == "bf16":
        from .rounding import round_bf16
        v = round_bf16(vals)
    ul, inv = np.unique(rows, return_inverse=True)
    order = np.argsort(inv, kind="stable")
    inv_s, cols_s, v_s = inv[order], cols[order], v[order]
    bounds = np.searchsorted(inv_s, np.arange(0, ul.size + row_chunk, row_chunk))
    XtT = Xt.T                     # n x k view: one row per column of X
    for c, r0 in enumerate(range(0, ul.size, row_chunk)):
        r1 = min(ul.size, r0 + row_chunk)
        P = pi_columns(seed, k, d, ul[r0:r1], kind, fmt)              # k x (r1 - r0)
        e0, e1 = bounds[c], bounds[c + 1]
        contrib = P[:, inv_s[e0:e1] - r0].T * v_s[e0:e1, None]         # one row v Pi[:, l] per triple
        np.add.at(XtT, cols_s[e0:e1], contrib)
    return Xt, nx2


def sketch_pair(a_entries, b_entries, d, n1, n2, seed, k, kind="gaussian", fmt=None):
    """(At, Bt, na2, nb2) as ``oracle.sketch.sketch`` returns them, for A and B
    given as (rows, cols, vals) triples; b_entries None is the A = B case."""
    At, na2 = sketch_entries(*a_entries, d, n1, seed, k, kind, fmt)
    if b_entries is None:
        return At, At, na2, na2
    Bt, nb2 = sketch_entries(*b_entries, d, n2, seed, k, kind, fmt)
    return At, Bt, na2, nb2

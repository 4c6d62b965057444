"""The subsampled randomized Hadamard transform as the sketching matrix
(Section 4, "Spark implementation": the paper's implementation sketched with
SRHT, which Section 2 "Step 1" admits as an oblivious subspace embedding).
Test infrastructure, like the rest of this package.

Definition (read from the SRHT's standard form Pi = sqrt(D/k) R H S; the
paper names the transform only):
  D       = the smallest power of two >= d (A and B padded with zero rows);
  S       = diag(sigma), sigma_l = +1 or -1 from bit 0 of the Philox word that
            the counter spec assigns to (row 0, column l) under tag 7;
  H       = the D x D Walsh-Hadamard matrix scaled by 1/sqrt(D),
            H[rho, l] = (-1)^popcount(rho & l) / sqrt(D) (Sylvester's order);
  R       = k rows rho_0 .. rho_{k-1} of H drawn uniformly with replacement,
            rho_c = the low log2(D) bits of the tag-8 word of (row 0, column c);
  Pi[c,l] = sqrt(D/k) H[rho_c, l] sigma_l = sigma_l (-1)^popcount(rho_c & l) / sqrt(k).
E[Pi^T Pi] = I, as for the Gaussian Pi. The oracle forms Pi block by block and
multiplies (the plain definition); the GPU computes the same product by fast
Walsh-Hadamard transforms of row chunks.
"""

import numpy as np

from .philox import stream_word_at

TAG_SRHT_SIGN = 7
TAG_SRHT_ROW = 8


def padded_size(d):
    """D: the smallest power of two >= d."""
    D = 1
    while D < d:
        D *= 2
    return D


def signs_at(seed, l):
    """sigma_l for an array of indices l as +1.0 / -1.0."""
    l = np.asarray(l, dtype=np.int64)
    w = stream_word_at(seed, TAG_SRHT_SIGN, np.zeros_like(l), l)
    return 1.0 - 2.0 * (w & 1).astype(np.float64)


def signs(seed, l0, l1):
    """sigma_l for l in [l0, l1) as +1.0 / -1.0."""
    return signs_at(seed, np.arange(l0, l1, dtype=np.int64))


def rows(seed, k, D):
    """rho_c for c < k: rows of H drawn uniformly with replacement."""
    c = np.arange(k, dtype=np.int64)
    w = stream_word_at(seed, TAG_SRHT_ROW, np.zeros_like(c), c).astype(np.int64)
    return w & (D - 1)


def hadamard_signs(rho, l):
    """(-1)^popcount(rho & l) for all pairs (rho x l), as +1.0 / -1.0."""
    x = np.bitwise_and(np.asarray(rho, dtype=np.int64)[:, None], np.asarray(l, dtype=np.int64)[None, :])
    par = np.zeros(x.shape, dtype=np.int64)
    while np.any(x):
        par ^= x & 1
        x >>= 1
    return 1.0 - 2.0 * par.astype(np.float64)


def pi_block(seed, k, d, l0, l1):
    """Pi[:, l0:l1] (k x (l1 - l0))."""
    rho = rows(seed, k, padded_size(d))
    l = np.arange(l0, l1, dtype=np.int64)
    return hadamard_signs(rho, l) * signs(seed, l0, l1)[None, :] / np.sqrt(float(k))


def pi_columns(seed, k, d, l):
    """Pi[:, l] (k x len(l)) for an array of indices l < d in any order."""
    l = np.asarray(l, dtype=np.int64)
    rho = rows(seed, k, padded_size(d))
    return hadamard_signs(rho, l) * signs_at(seed, l)[None, :] / np.sqrt(float(k))


def sketch(A, B, seed, k, chunk=4096):
    """The single pass with the SRHT: (At, Bt, na2, nb2) as oracle.sketch.sketch
    returns them (B None: the A = B case)."""
    A = np.asarray(A)
    d, n1 = A.shape
    same = B is None
    if not same:
        B = np.asarray(B)
    n2 = n1 if same else B.shape[1]
    At = np.zeros((k, n1))
    Bt = None if same else np.zeros((k, n2))
    na2 = np.zeros(n1)
    nb2 = None if same else np.zeros(n2)
    for l0 in range(0, d, chunk):
        l1 = min(d, l0 + chunk)
        P = pi_block(seed, k, d, l0, l1)
        a = np.asarray(A[l0:l1], dtype=np.float64)
        At += P @ a
        na2 += np.einsum("li,li->i", a, a)
        if not same:
            b = np.asarray(B[l0:l1], dtype=np.float64)
            Bt += P @ b
            nb2 += np.einsum("li,li->i", b, b)
    if same:
        return At, At, na2, na2
    return At, Bt, na2, nb2

"""One pass over A and B (Alg. 1 step 2; Section 2, "Step 1").

Computes the Gaussian JL sketches A~ = Pi A (k x n1), B~ = Pi B (k x n2) with
Pi(c, l) ~ N(0, 1/k) i.i.d., and the exact squared column norms ||A_i||^2,
||B_j||^2. Everything is FP64. The pass is chunked over the d rows only to
bound memory; a chunk of rows of Pi is produced from the counter spec (see
``oracle.philox``) exactly as the whole matrix would be.

Pi(c, l) = Z(c, l) / sqrt(k), Z(c, l) = lane (c mod 4) of the Box-Muller
variates of Philox(seed; counter = (c // 4, l mod 2^32, TAG_PI, l >> 32)).
"""

import numpy as np

from .philox import TAG_PI, stream_words
from .gaussian import normals_from_words


def gaussian_block(seed, k, l0, l1):
    """Z[:, l0:l1] (k x (l1-l0)) of i.i.d. N(0,1) variates, FP64."""
    nb = (k + 3) // 4
    rows = np.arange(l0, l1, dtype=np.int64)[:, None]
    cbs = np.arange(nb, dtype=np.int64)[None, :]
    w = stream_words(seed, TAG_PI, rows, cbs)                # each (W, nb)
    z = np.stack(normals_from_words(*w), axis=-1)            # (W, nb, 4)
    z = z.reshape(l1 - l0, 4 * nb)[:, :k]                    # (W, k): column c is lane c%4 of block c//4
    return np.ascontiguousarray(z.T)


def pi_block(seed, k, l0, l1):
    """Pi[:, l0:l1] = Z / sqrt(k): entries N(0, 1/k) (Alg. 1 step 2)."""
    return gaussian_block(seed, k, l0, l1) / np.sqrt(float(k))


def sketch(A, B, seed, k, chunk=8192):
    """Single pass: returns (At, Bt, na2, nb2).

    A: d x n1, B: d x n2 (any real dtype; widened to FP64) or None for the
    A = B case (Section 3, Remark 3), in which case Bt is At and nb2 is na2.
    At = Pi A (k x n1), Bt = Pi B (k x n2), na2[i] = ||A_i||^2, nb2[j] = ||B_j||^2.
    """
    A = np.asarray(A)
    d, n1 = A.shape
    same = B is None
    if not same:
        B = np.asarray(B)
        assert B.shape[0] == d
    n2 = n1 if same else B.shape[1]
    At = np.zeros((k, n1))
    Bt = None if same else np.zeros((k, n2))
    na2 = np.zeros(n1)
    nb2 = None if same else np.zeros(n2)
    for l0 in range(0, d, chunk):
        l1 = min(d, l0 + chunk)
        P = pi_block(seed, k, l0, l1)
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


def sketch_with_pi(Pi, A, B):
    """The same pass with an explicit sketching matrix Pi (k x d). Any oblivious
    subspace embedding is admissible (Section 2, "Step 1"); tests use it to
    inject Pi = I or an orthonormal Pi."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    return Pi @ A, Pi @ B, (A * A).sum(axis=0), (B * B).sum(axis=0)


def sketch_lowp(A, B, seed, k, fmt, chunk=8192):
    """The pass with the GEMM operands in a narrow format (no precision is
    fixed by the paper; Alg. 1 step 2 forms Pi A and Pi B). Definition:
    At = (1/sqrt(k)) R(Z) R(A), Bt = (1/sqrt(k)) R(Z) R(B) with R the rounding
    of every entry to `fmt` (``oracle.rounding``) and the product exact (FP64
    here). The squared column norms are those of the unrounded data.
    fmt: "bf16" (both operands rounded to bfloat16) or "fp8" (Pi rounded to
    E4M3; the data to E4M3 with one E8M0 scale per column and block of 32
    global rows, see ``oracle.rounding.quantize_e4m3_blocks``; chunk is then
    a multiple of 32). Same return convention as ``sketch``."""
    from .rounding import quantize_e4m3_blocks, round_bf16, round_e4m3
    if fmt == "bf16":
        rnd_pi, rnd_x = round_bf16, lambda a, l0: round_bf16(a)
    elif fmt == "fp8":
        chunk = max(32, chunk // 32 * 32)
        rnd_pi, rnd_x = round_e4m3, quantize_e4m3_blocks
    else:
        raise ValueError(f"unknown format {fmt!r}")
    A = np.asarray(A)
    d, n1 = A.shape
    same = B is None
    if not same:
        B = np.asarray(B)
        assert B.shape[0] == d
    n2 = n1 if same else B.shape[1]
    At = np.zeros((k, n1))
    Bt = None if same else np.zeros((k, n2))
    na2 = np.zeros(n1)
    nb2 = None if same else np.zeros(n2)
    for l0 in range(0, d, chunk):
        l1 = min(d, l0 + chunk)
        Z = rnd_pi(gaussian_block(seed, k, l0, l1))
        a = np.asarray(A[l0:l1], dtype=np.float64)
        At += Z @ rnd_x(a, l0)
        na2 += np.einsum("li,li->i", a, a)
        if not same:
            b = np.asarray(B[l0:l1], dtype=np.float64)
            Bt += Z @ rnd_x(b, l0)
            nb2 += np.einsum("li,li->i", b, b)
    At /= np.sqrt(float(k))
    if same:
        return At, At, na2, na2
    Bt /= np.sqrt(float(k))
    return At, Bt, na2, nb2

"""Evaluation (Section 4): the spectral-norm error ||A^T B - X|| / ||A^T B|| of a
rank-r approximation X, and the best achievable value ("Optimal" in Table 1),
sigma_{r+1}(A^T B) / sigma_1(A^T B) by the Eckart-Young theorem.

A^T B is formed exactly in FP64 (the naive O(n^2 d) product of Section 1); it
is the ground truth the method is measured against and never part of the method.
"""

import numpy as np
import scipy.linalg
import scipy.sparse.linalg


def product(A, B, chunk=16384):
    """A^T B in FP64, accumulated over chunks of the d rows. B=None means A^T A."""
    A = np.asarray(A)
    d = A.shape[0]
    Bm = A if B is None else np.asarray(B)
    out = np.zeros((A.shape[1], Bm.shape[1]))
    for l0 in range(0, d, chunk):
        a = np.asarray(A[l0:l0 + chunk], dtype=np.float64)
        b = a if B is None else np.asarray(Bm[l0:l0 + chunk], dtype=np.float64)
        out += a.T @ b
    return out


def spectral_norm(M):
    """Largest singular value of a dense matrix (LAPACK for small, ARPACK above)."""
    M = np.asarray(M, dtype=np.float64)
    if min(M.shape) <= 1500:
        return float(scipy.linalg.svdvals(M)[0])
    return float(scipy.sparse.linalg.svds(M, k=1, return_singular_vectors=False, tol=1e-12)[0])


def singular_values(M, count):
    """The top `count` singular values of M, descending."""
    M = np.asarray(M, dtype=np.float64)
    if min(M.shape) <= 1500 or count >= min(M.shape) - 1:
        return scipy.linalg.svdvals(M)[:count]
    s = scipy.sparse.linalg.svds(M, k=count, return_singular_vectors=False, tol=1e-12)
    return np.sort(s)[::-1]


def relative_error(AtB, U, sigma, V):
    """||A^T B - U diag(sigma) V^T||_2 / ||A^T B||_2 (sigma=None: U V^T)."""
    X = (U * sigma[None, :]) @ V.T if sigma is not None else U @ V.T
    return spectral_norm(AtB - X) / spectral_norm(AtB)


def optimal_error(AtB, r):
    """sigma_{r+1} / sigma_1 of A^T B: the error of the best rank-r approximation."""
    s = singular_values(AtB, r + 1)
    return float(s[r] / s[0])

"""Weighted alternating minimisation, WAltMin (Appendix A, Alg. 2).

  R_Omega(X)     = w .* P_Omega(X)                          (Appendix A, definition)
  init           U0 S0 V0^T = rank-r SVD of R_Omega0(M~)   (Alg. 2 steps 4-5)
  trim           zero row i of U0 if ||U0_i|| > 8 sqrt(r) ||A_i|| / ||A||_F
                 (Alg. 2 step 6; the bound is the one stated for the trimmed
                 iterate in Appendix C, proof of Lemma B.7's corollary)
  for t = 0 .. T-1                                          (Alg. 2 steps 7-10)
     V^(t+1) = argmin_V || R^{1/2}_{Omega_{2t+1}} (M~ - U^(t) V^T) ||_F^2
     U^(t+1) = argmin_U || R^{1/2}_{Omega_{2t+2}} (M~ - U V^(t+1)^T) ||_F^2

Each argmin separates into one weighted least-squares problem per column j
(resp. row i): minimise sum_i w_ij (q_i^T v - M~_ij)^2, whose normal equations
are G_j v = h_j with G_j = sum_i w_ij q_i q_i^T and h_j = sum_i w_ij M~_ij q_i
(the rank-1 closed form of Appendix C, proof of Theorem 3.1, is the r = 1 case).

Readings where the paper is silent:
  * the fixed factor is orthonormalised (QR) before each half-step; the product
    U V^T is unchanged by this, only the conditioning improves;
  * no regularisation; G is factored by an explicit Cholesky; a pivot (diagonal
    entry before the square root) <= 1e-12 * max diag(G) is a failure, after which
    the factorisation is retried once on G + 1e-9 * trace(G)/r * I (a ridge term
    large enough to clear the pivot test, so a rank-deficient G yields the
    near-minimum-norm solution); if that also fails, or the row/column has no
    samples, its solution is 0;
  * REUSE mode uses Omega for every subset (the sample is not split); SPLIT mode
    uses the 2T+1 subsets drawn by oracle.sample;
  * T = 0 returns the trimmed initial factors U0 S0 and V0;
  * output: U = U^(T) (solved against the orthonormalised V^(T)) and that
    orthonormal V; the canonical form is U = Q_U X, V = Q_V Y, sigma from
    the SVD X diag(sigma) Y^T of the r x r factor R_U of U = Q_U R_U.
"""

import numpy as np
import scipy.sparse as sp

REL_PIVOT = 1e-12
RETRY_SHIFT = 1e-9


def _cholesky(G, rel_tol):
    """Batched explicit Cholesky G_b = L_b L_b^T, column by column, sums taken
    sequentially in index order. Returns (L, ok)."""
    nb, r, _ = G.shape
    L = np.zeros_like(G)
    maxdiag = np.max(np.diagonal(G, axis1=1, axis2=2), axis=1) if r else np.zeros(nb)
    tol = rel_tol * maxdiag
    ok = maxdiag > 0
    for j in range(r):
        s = G[:, j, j].copy()
        for k in range(j):
            s = s - L[:, j, k] * L[:, j, k]
        ok &= s > tol
        djj = np.sqrt(np.where(ok, s, 1.0))
        L[:, j, j] = djj
        for i in range(j + 1, r):
            t = G[:, i, j].copy()
            for k in range(j):
                t = t - L[:, i, k] * L[:, j, k]
            L[:, i, j] = t / djj
    return L, ok


def _tri_solve(L, h):
    """Solve L L^T x = h for each batch entry (forward then back substitution)."""
    nb, r, _ = L.shape
    y = np.zeros((nb, r))
    for i in range(r):
        t = h[:, i].copy()
        for k in range(i):
            t = t - L[:, i, k] * y[:, k]
        y[:, i] = t / L[:, i, i]
    x = np.zeros((nb, r))
    for i in range(r - 1, -1, -1):
        t = y[:, i].copy()
        for k in range(i + 1, r):
            t = t - L[:, k, i] * x[:, k]
        x[:, i] = t / L[:, i, i]
    return x


def chol_solve(G, h, rel_pivot=REL_PIVOT):
    """Solve the batch of r x r systems G_b x_b = h_b with the pivot rule above."""
    G = np.asarray(G, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    nb, r, _ = G.shape
    x = np.zeros((nb, r))
    L, ok = _cholesky(G, rel_pivot)
    if ok.any():
        x[ok] = _tri_solve(L[ok], h[ok])
    bad = ~ok
    maxdiag = np.max(np.diagonal(G, axis1=1, axis2=2), axis=1) if r else np.zeros(nb)
    retry = bad & (maxdiag > 0)
    if retry.any():
        Gr = G[retry].copy()
        shift = RETRY_SHIFT * np.trace(Gr, axis1=1, axis2=2) / r
        Gr = Gr + shift[:, None, None] * np.eye(r)[None]
        L2, ok2 = _cholesky(Gr, rel_pivot)
        xr = np.zeros((Gr.shape[0], r))
        if ok2.any():
            xr[ok2] = _tri_solve(L2[ok2], h[retry][ok2])
        x[retry] = xr
    return x


def normal_equations(out_idx, in_idx, w, mt, n_out, Q):
    """G (n_out x r x r) and h (n_out x r) of the per-row least-squares problems.

    Entry e couples output index out_idx[e] with input index in_idx[e]:
      G[o] = sum_e w_e Q[in_e] Q[in_e]^T,  h[o] = sum_e w_e mt_e Q[in_e].
    """
    n_in, r = Q.shape
    Sw = sp.csr_matrix((w, (out_idx, in_idx)), shape=(n_out, n_in))
    Swm = sp.csr_matrix((w * mt, (out_idx, in_idx)), shape=(n_out, n_in))
    G = np.empty((n_out, r, r))
    for a in range(r):
        G[:, a, :] = Sw @ (Q * Q[:, a:a + 1])
    h = Swm @ Q
    return G, h


def orthonormalize(X):
    """Q factor of a thin QR (Householder, LAPACK) of X."""
    Q, _ = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    return Q


def init(n1, n2, rows, cols, w, mt, r, na2, FA):
    """Alg. 2 steps 4-6: rank-r SVD of R_Omega0(M~) (densified), then trim.
    Returns (U0_trimmed, S0, V0, trimmed_mask)."""
    R0 = np.zeros((n1, n2))
    R0[rows, cols] = w * mt
    U, s, Vt = np.linalg.svd(R0, full_matrices=False)
    U0, S0, V0 = U[:, :r].copy(), s[:r].copy(), Vt[:r].T.copy()
    thresh = 8.0 * np.sqrt(r) * np.sqrt(np.asarray(na2, dtype=np.float64) / FA) if FA > 0 else np.zeros(n1)
    trimmed = np.linalg.norm(U0, axis=1) > thresh
    U0[trimmed] = 0.0
    return U0, S0, V0, trimmed


def waltmin(n1, n2, rows, cols, w, mt, r, T, na2, FA, subset=None):
    """Alg. 2. rows, cols, w, mt list Omega with weights and M~ values; subset
    (SPLIT mode) gives each entry's subset in [0, 2T]; None means REUSE.
    Returns dict(U, V, U0, S0, V0, trimmed)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    mt = np.asarray(mt, dtype=np.float64)

    def pick(s):
        if subset is None:
            return slice(None)
        return subset == s

    p0 = pick(0)
    U0, S0, V0, trimmed = init(n1, n2, rows[p0], cols[p0], w[p0], mt[p0], r, na2, FA)
    if T == 0:
        return dict(U=U0 * S0[None, :], V=V0, U0=U0, S0=S0, V0=V0, trimmed=trimmed)
    Uh = U0
    Qv = None
    for t in range(T):
        Qu = orthonormalize(Uh)
        pv = pick(2 * t + 1)
        G, h = normal_equations(cols[pv], rows[pv], w[pv], mt[pv], n2, Qu)
        Vh = chol_solve(G, h)
        Qv = orthonormalize(Vh)
        pu = pick(2 * t + 2)
        G, h = normal_equations(rows[pu], cols[pu], w[pu], mt[pu], n1, Qv)
        Uh = chol_solve(G, h)
    return dict(U=Uh, V=Qv, U0=U0, S0=S0, V0=V0, trimmed=trimmed)


def canonical(U, V):
    """Canonical SVD form of U V^T: orthonormal Uc, Vc and sigma with
    U V^T = Uc diag(sigma) Vc^T. Each component's sign makes the entry of
    largest magnitude of its Vc column positive."""
    Qu, Ru = np.linalg.qr(U, mode="reduced")
    Qv, Rv = np.linalg.qr(V, mode="reduced")
    X, s, Yt = np.linalg.svd(Ru @ Rv.T)
    Uc, Vc = Qu @ X, Qv @ Yt.T
    for c in range(Vc.shape[1]):
        if Vc[np.argmax(np.abs(Vc[:, c])), c] < 0:
            Uc[:, c] *= -1
            Vc[:, c] *= -1
    return Uc, s, Vc

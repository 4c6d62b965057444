"""Pins for the oracle's WAltMin (Appendix A, Alg. 2), evaluation (Section 4)
and the whole pipeline (Alg. 1)."""

import math

import numpy as np
import pytest

from oracle import sketch, sample, estimate, waltmin, evaluate, solve
import smp_inputs


# ---------------------------------------------------------------- solves

def test_chol_solve_matches_lapack():
    rng = np.random.default_rng(0)
    for r in (1, 5, 10, 20):
        X = rng.standard_normal((64, 3 * r, r))
        G = np.einsum("bki,bkj->bij", X, X)
        h = rng.standard_normal((64, r))
        x = waltmin.chol_solve(G, h)
        assert np.allclose(x, np.linalg.solve(G, h[..., None])[..., 0], rtol=1e-9, atol=1e-12)


def test_chol_pivot_rule():
    # no samples -> zero; rank-deficient -> shifted retry gives a finite solution
    G = np.zeros((3, 2, 2))
    G[1] = [[1.0, 1.0], [1.0, 1.0]]                  # singular
    G[2] = [[4.0, 0.0], [0.0, 1e-20]]                # pivot far below 1e-12 * max diag
    h = np.array([[1.0, 1.0], [2.0, 2.0], [4.0, 0.0]])
    x = waltmin.chol_solve(G, h)
    assert np.all(x[0] == 0.0)
    Gs = G[1] + 1e-9 * 2.0 / 2 * np.eye(2)
    assert np.allclose(x[1], np.linalg.solve(Gs, h[1]), rtol=1e-6)
    assert np.allclose(x[1], [1.0, 1.0], rtol=1e-6)            # minimum-norm solution
    assert np.allclose(x[2], [1.0, 0.0])


def test_weighted_least_squares_equals_lstsq():
    """One half-step is, per column j, the weighted least-squares problem
    min_v sum_i w_ij (q_i^T v - M~_ij)^2 (Alg. 2 step 8), i.e. ordinary least
    squares on the rows scaled by sqrt(w)."""
    rng = np.random.default_rng(4)
    n1, n2, r = 40, 7, 3
    Q, _ = np.linalg.qr(rng.standard_normal((n1, r)))
    mask = rng.random((n1, n2)) < 0.5
    rows, cols = np.nonzero(mask)
    w = 1.0 / rng.uniform(0.1, 1.0, rows.size)
    mt = rng.standard_normal(rows.size)
    G, h = waltmin.normal_equations(cols, rows, w, mt, n2, Q)
    V = waltmin.chol_solve(G, h)
    for j in range(n2):
        sel = cols == j
        sw = np.sqrt(w[sel])
        ref = np.linalg.lstsq(Q[rows[sel]] * sw[:, None], mt[sel] * sw, rcond=None)[0]
        assert np.allclose(V[j], ref, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------- WAltMin

def _full_problem(A, B, r, T):
    """Every entry observed with q^ = 1 and exact values M~ = A^T B."""
    n1, n2 = A.shape[1], B.shape[1]
    rows, cols = [a.ravel() for a in np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")]
    M = A.T @ B
    na2 = (A * A).sum(0)
    return waltmin.waltmin(n1, n2, rows, cols, np.ones(rows.size), M[rows, cols], r, T, na2, 1e-300)  # tiny F_A: trim threshold never reached


def test_full_observation_is_eckart_young():
    """All q^ = 1 and M~ = A^T B (k = d, orthonormal Pi): WAltMin returns the
    best rank-r approximation (A^T B)_r, already after the first iteration."""
    rng = np.random.default_rng(2)
    A = rng.standard_normal((50, 30))
    B = rng.standard_normal((50, 25))
    M = A.T @ B
    U, s, Vt = np.linalg.svd(M)
    Mr = (U[:, :4] * s[:4]) @ Vt[:4]
    res = _full_problem(A, B, 4, 1)
    assert np.allclose(res["U"] @ res["V"].T, Mr, atol=1e-10 * s[0])
    res0 = _full_problem(A, B, 4, 0)
    assert np.allclose(res0["U"] @ res0["V"].T, Mr, atol=1e-10 * s[0])


def test_exact_low_rank_recovered_from_samples():
    """A^T B of rank r, exact entries on a sample above the phase transition
    (m = 4 n r log n, Section 4): WAltMin recovers A^T B (the error bound of
    Theorem 3.1 vanishes for rank-r A^T B)."""
    rng = np.random.default_rng(5)
    d, n, r = 100, 120, 3
    Z = rng.standard_normal((d, r))
    A = Z @ rng.standard_normal((r, n))
    B = Z @ rng.standard_normal((r, n))
    na2, nb2 = (A * A).sum(0), (B * B).sum(0)
    m = 4 * n * r * math.log(n)
    om = sample.sample(na2, nb2, m, seed=3)
    M = A.T @ B
    res = waltmin.waltmin(n, n, om.rows, om.cols, om.w, M[om.rows, om.cols], r, 30, na2, om.FA)
    X = res["U"] @ res["V"].T
    assert np.linalg.norm(X - M, 2) / np.linalg.norm(M, 2) < 1e-8


def test_trim_zeroes_spiky_rows():
    """Alg. 2 step 6: rows of U0 above 8 sqrt(r) ||A_i|| / ||A||_F are zeroed."""
    n1, n2, r = 20, 20, 2
    M = np.zeros((n1, n2))
    M[0, 0] = 100.0                  # one spike dominates the SVD
    M[1:, 1:] = np.random.default_rng(0).standard_normal((19, 19)) * 0.01
    rows, cols = [a.ravel() for a in np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")]
    na2 = np.ones(n1)
    na2[0] = 1e-6                    # but A_0 itself is tiny
    U0, S0, V0, trimmed = waltmin.init(n1, n2, rows, cols, np.ones(rows.size), M.ravel(), r, na2, na2.sum())
    assert trimmed[0] and np.all(U0[0] == 0.0)
    assert trimmed.sum() == 1


def test_product_invariant_to_orthonormalisation():
    """Solving against U R instead of U changes V to V R^{-T}; the product is
    unchanged (why orthonormalising the fixed factor is harmless)."""
    rng = np.random.default_rng(6)
    n1, n2, r = 30, 20, 3
    rows, cols = np.nonzero(rng.random((n1, n2)) < 0.6)
    w = rng.uniform(1, 3, rows.size)
    mt = rng.standard_normal(rows.size)
    U = rng.standard_normal((n1, r))
    R = np.triu(rng.standard_normal((r, r))) + 3 * np.eye(r)
    G, h = waltmin.normal_equations(cols, rows, w, mt, n2, U)
    V1 = waltmin.chol_solve(G, h)
    G, h = waltmin.normal_equations(cols, rows, w, mt, n2, U @ R)
    V2 = waltmin.chol_solve(G, h)
    assert np.allclose(U @ V1.T, (U @ R) @ V2.T, rtol=1e-9, atol=1e-12)


def test_canonical_form():
    rng = np.random.default_rng(8)
    U, V = rng.standard_normal((15, 4)), rng.standard_normal((11, 4))
    Uc, s, Vc = waltmin.canonical(U, V)
    assert np.allclose((Uc * s) @ Vc.T, U @ V.T, atol=1e-12)
    assert np.allclose(Uc.T @ Uc, np.eye(4), atol=1e-12) and np.allclose(Vc.T @ Vc, np.eye(4), atol=1e-12)
    assert np.all(np.diff(s) <= 0)
    assert np.allclose(s, np.linalg.svd(U @ V.T, compute_uv=False)[:4])


# ---------------------------------------------------------------- evaluation

def test_optimal_error_is_eckart_young():
    rng = np.random.default_rng(9)
    M = rng.standard_normal((40, 30))
    U, s, Vt = np.linalg.svd(M)
    r = 5
    e = evaluate.relative_error(M, U[:, :r], s[:r], Vt[:r].T)
    assert abs(e - evaluate.optimal_error(M, r)) < 1e-12
    assert abs(e - s[r] / s[0]) < 1e-12


def test_product_is_exact_over_many_chunks():
    """A^T B accumulated over several 16,384-row chunks with a ragged last
    chunk: on small-integer data every FP64 partial sum is an exact integer,
    so the result must equal the exact integer product (int64 arithmetic),
    for A^T B and for the A = B path."""
    rng = np.random.default_rng(12)
    d = 3 * 16384 + 517
    A = rng.integers(-8, 9, size=(d, 30)).astype(np.float32)
    B = rng.integers(-8, 9, size=(d, 23)).astype(np.float32)
    Ai, Bi = A.astype(np.int64), B.astype(np.int64)
    got = evaluate.product(A, B)
    assert np.array_equal(got, (Ai.T @ Bi).astype(np.float64))
    assert np.array_equal(evaluate.product(A, None), (Ai.T @ Ai).astype(np.float64))
    # dropping or repeating any chunk changes the exact result
    assert not np.array_equal(got, (Ai[16384:].T @ Bi[16384:]).astype(np.float64))


def test_spectral_norm_large_path_matches_lapack():
    M = np.random.default_rng(1).standard_normal((1600, 1501))
    import scipy.linalg
    assert abs(evaluate.spectral_norm(M) / scipy.linalg.svdvals(M)[0] - 1) < 1e-10


# ---------------------------------------------------------------- pipeline

def _c1_like(seed, d=1000, n=120, R=4):
    A, B = smp_inputs.latent_pair(d, n, n, R, 0.1, 0.5, seed)
    return A.numpy(), B.numpy()


def test_pipeline_k_equal_d_orthonormal_is_near_optimal():
    """With exact estimates (orthonormal Pi, k = d) and m above the phase
    transition the pipeline reaches the optimal rank-r error."""
    A, B = _c1_like(1, d=150, n=100, R=3)
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((150, 150)))
    At, Bt, na2, nb2 = sketch.sketch_with_pi(Q, A, B)
    om = sample.sample(na2, nb2, 4 * 100 * 3 * math.log(100), seed=2)
    mt = estimate.estimate(At, Bt, na2, nb2, om.rows, om.cols)
    res = waltmin.waltmin(100, 100, om.rows, om.cols, om.w, mt, 3, 10, na2, om.FA)
    AtB = evaluate.product(A, B)
    e = evaluate.relative_error(AtB, res["U"], None, res["V"])
    e_opt = evaluate.optimal_error(AtB, 3)
    assert e < max(3 * e_opt, 1e-3)


def test_pipeline_error_ordering_and_trend_in_k():
    """e_opt <= e, and the error decreases as the sketch size k grows
    (Section 4, comparison with LELA; Theorem 3.1). Averaged over seeds."""
    A, B = _c1_like(3)
    AtB = evaluate.product(A, B)
    e_opt = evaluate.optimal_error(AtB, 4)
    m = solve.default_m(120, 120, 4)
    errs = {}
    for k in (20, 80, 320):
        es = []
        for s in range(3):
            res = solve.smp_pca(A, B, 4, k, m, 10, seed=100 + s)
            es.append(evaluate.relative_error(AtB, res["Uc"], res["sigma"], res["Vc"]))
        errs[k] = np.mean(es)
        assert min(es) >= e_opt
    assert errs[20] > errs[80] > errs[320]


def test_pipeline_beats_svd_of_sketch_product_on_cone():
    """Figure 4(b): for columns from a narrow cone, SMP-PCA's error is far below
    that of the rank-r SVD of A~^T B~."""
    A, B = smp_inputs.cone_pair(500, 100, 0.3, 7)
    A, B = A.numpy(), B.numpy()
    AtB = evaluate.product(A, B)
    res = solve.smp_pca(A, B, 2, 20, 1e9, 10, seed=5)       # all entries sampled
    e_smp = evaluate.relative_error(AtB, res["Uc"], res["sigma"], res["Vc"])
    U, s, Vt = np.linalg.svd(res["At"].T @ res["Bt"])
    e_svd = evaluate.relative_error(AtB, U[:, :2], s[:2], Vt[:2].T)
    assert e_smp < 0.5 * e_svd


def test_split_mode_uses_fresh_subsets():
    """Alg. 2 step 3 (SPLIT mode): 2T+1 subsets, init on Omega_0, the half-steps
    on Omega_1 .. Omega_2T. With exact rank-r entries and every entry observed,
    each subset holds ~1/(2T+1) of the grid and the iterates still approach
    A^T B; changing the values on Omega_0 moves the init."""
    rng = np.random.default_rng(5)
    d, n, r, T = 100, 120, 3, 2
    Z = rng.standard_normal((d, r))
    A = Z @ rng.standard_normal((r, n))
    B = Z @ rng.standard_normal((r, n))
    na2, nb2 = (A * A).sum(0), (B * B).sum(0)
    om = sample.sample(na2, nb2, 1e12, seed=3, T=T, split=True)
    assert om.nnz == n * n and set(np.unique(om.subset)) == set(range(2 * T + 1))
    M = A.T @ B
    vals = M[om.rows, om.cols]
    res = waltmin.waltmin(n, n, om.rows, om.cols, om.w, vals, r, T, na2, om.FA, subset=om.subset)
    X = res["U"] @ res["V"].T
    assert np.linalg.norm(X - M, 2) / np.linalg.norm(M, 2) < 0.1
    noisy = vals.copy()
    noisy[om.subset == 0] += rng.standard_normal((om.subset == 0).sum())
    res3 = waltmin.waltmin(n, n, om.rows, om.cols, om.w, noisy, r, T, na2, om.FA, subset=om.subset)
    assert not np.allclose(res3["U0"], res["U0"])         # init reads Omega_0


def test_pipeline_a_equals_b_pca():
    """Section 3, Remark 3: A = B computes a rank-r approximation of A^T A."""
    A, _ = _c1_like(5)
    AtA = evaluate.product(A, None)
    res = solve.smp_pca(A, None, 4, 200, solve.default_m(120, 120, 4), 10, seed=3)
    assert res["At"] is res["Bt"]
    e = evaluate.relative_error(AtA, res["Uc"], res["sigma"], res["Vc"])
    assert e < 0.1


def test_empty_omega_gives_zero_approximation():
    """Degenerate case of Alg. 1: with no sampled entry R_Omega(M~) is the zero
    matrix, so the rank-r fit of Alg. 2 is zero (sigma = 0) and every
    least-squares row has no equations (zero solution)."""
    A, B = smp_inputs.latent_pair(500, 50, 60, 3, 0.1, 0.5, 7)
    A, B = A.numpy(), B.numpy()
    res = solve.smp_pca(A, B, 3, 20, 1e-6, 4, seed=7)
    assert res["omega"].nnz == 0
    assert np.array_equal(res["sigma"], np.zeros(3))
    assert np.all(np.isfinite(res["Uc"])) and np.all(np.isfinite(res["Vc"]))
    assert not np.any(res["U"])                            # no equations: zero rows

"""Pins for the oracle's one-pass sketch (Alg. 1 step 2), sampling (Eq. (1),
Alg. 1 step 3) and rescaled-JL estimator (Eq. (2))."""

import math

import numpy as np
import pytest
import scipy.stats

from oracle import sketch, sample, estimate


def _mats(d=300, n1=17, n2=23, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, n1)) * (np.arange(1, n1 + 1) ** -0.5)
    B = rng.standard_normal((d, n2)) * (np.arange(1, n2 + 1) ** -0.7)
    return A, B


# ---------------------------------------------------------------- sketch

def test_identity_pi_reproduces_inputs():
    A, B = _mats(d=40)
    At, Bt, na2, nb2 = sketch.sketch_with_pi(np.eye(40), A, B)
    assert np.array_equal(At, A) and np.array_equal(Bt, B)
    assert np.allclose(na2, np.linalg.norm(A, axis=0) ** 2, rtol=1e-14)


def test_orthonormal_pi_preserves_products():
    """Lemma B.1 with no distortion: an orthogonal Pi (k = d) keeps A^T B."""
    A, B = _mats(d=60)
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((60, 60)))
    At, Bt, _, _ = sketch.sketch_with_pi(Q, A, B)
    assert np.allclose(At.T @ Bt, A.T @ B, atol=1e-12 * np.abs(A.T @ B).max())


def test_sketch_norms_are_library_column_norms():
    A, B = _mats(d=5000, n1=9, n2=4)
    At, Bt, na2, nb2 = sketch.sketch(A, B, seed=5, k=8, chunk=777)
    assert np.allclose(na2, np.linalg.norm(A, axis=0) ** 2, rtol=1e-13)
    assert np.allclose(nb2, np.linalg.norm(B, axis=0) ** 2, rtol=1e-13)


def test_sketch_independent_of_chunking_and_equals_pi_times_a():
    A, B = _mats(d=1000)
    At1, Bt1, _, _ = sketch.sketch(A, B, seed=9, k=13, chunk=1000)
    At2, Bt2, _, _ = sketch.sketch(A, B, seed=9, k=13, chunk=97)
    assert np.allclose(At1, At2, rtol=1e-12, atol=1e-12)
    P = sketch.pi_block(9, 13, 0, 1000)
    assert np.allclose(At1, P @ A, atol=1e-12)
    assert np.allclose(Bt1, P @ B, atol=1e-12)


def test_pi_rows_are_prefix_stable_in_k():
    """Sketch row c depends on (seed, c, l) only, not on k."""
    P10 = sketch.gaussian_block(4, 10, 0, 50)
    P7 = sketch.gaussian_block(4, 7, 0, 50)
    assert np.array_equal(P10[:7], P7)


def test_sketch_is_unbiased_for_gram():
    """E[A~^T B~] = A^T B for Pi with i.i.d. N(0, 1/k) entries (JL property)."""
    A, B = _mats(d=80, n1=3, n2=3)
    acc = np.zeros((3, 3))
    S = 400
    vals = []
    for s in range(S):
        At, Bt, _, _ = sketch.sketch(A, B, seed=500 + s, k=5)
        vals.append(At.T @ Bt)
    vals = np.array(vals)
    mean, sd = vals.mean(0), vals.std(0) / math.sqrt(S)
    assert np.all(np.abs(mean - A.T @ B) < 5 * sd + 1e-12)


def test_a_equals_b_case_shares_the_sketch():
    A, _ = _mats()
    At, Bt, na2, nb2 = sketch.sketch(A, None, seed=1, k=6)
    At2, Bt2, _, _ = sketch.sketch(A, A.copy(), seed=1, k=6)
    assert At is Bt and np.array_equal(At, At2) and np.array_equal(Bt2, At2)


# ---------------------------------------------------------------- sampling

def test_fixed_order_sum_matches_exact_sum():
    x = np.random.default_rng(2).random(1000) * 1e3
    assert abs(sample.fixed_order_sum(x) - math.fsum(x)) <= 1e-12 * math.fsum(x)
    # the order is sequential in blocks of 256 then over block sums
    blocks = [float(np.cumsum(x[b:b + 256])[-1]) for b in range(0, 1000, 256)]
    s = 0.0
    for b in blocks:
        s += b
    assert sample.fixed_order_sum(x) == s


def test_q_sums_to_m():
    """Eq. (1): sum_ij q_ij = m (the basis of 'roughly m samples')."""
    A, B = _mats()
    na2, nb2 = (A * A).sum(0), (B * B).sum(0)
    m = 123.4
    q = sample.probabilities(na2, nb2, m)
    assert abs(q.sum() - m) < 1e-12 * m


def test_q_row_sums_match_appendix_d():
    """App. D: the expected number of samples in row i is
    m (||A_i||^2 / (2 ||A||_F^2) + 1 / (2 n)) (n = n1 for the B-term)."""
    A, B = _mats()
    na2, nb2 = (A * A).sum(0), (B * B).sum(0)
    m = 50.0
    q = sample.probabilities(na2, nb2, m)
    mi = m * (na2 / (2 * na2.sum()) + 1.0 / (2 * A.shape[1]))
    assert np.allclose(q.sum(1), mi, rtol=1e-12)


def test_thresholds_exact_and_clamped():
    alpha = np.array([0.0, 0.25, 2.0])
    beta = np.array([0.0, 0.125])
    qhat, thr = sample.thresholds(alpha, beta, 1.0)
    assert qhat.max() == 1.0 and qhat.min() == 0.0
    assert thr[0, 0] == 0 and thr[1, 0] == 2**30 and thr[1, 1] == 3 * 2**29 and thr[2, 1] == 2**32


def test_sampling_frequencies_match_qhat():
    """Each entry is kept independently with probability q^ (Alg. 1 step 3)."""
    A, B = _mats(d=50, n1=6, n2=5)
    na2, nb2 = (A * A).sum(0), (B * B).sum(0)
    m = 12.0
    qhat = np.minimum(1, sample.probabilities(na2, nb2, m))
    S = 3000
    cnt = np.zeros_like(qhat)
    for s in range(S):
        om = sample.sample(na2, nb2, m, seed=10_000 + s)
        cnt[om.rows, om.cols] += 1
    freq = cnt / S
    sd = np.sqrt(qhat * (1 - qhat) / S) + 1e-12
    assert np.all(np.abs(freq - qhat) < 5 * sd + 1e-9)
    assert np.all(cnt[qhat == 1.0] == S)


def test_omega_size_and_weights():
    A, B = _mats(d=100, n1=200, n2=150)
    na2, nb2 = (A * A).sum(0), (B * B).sum(0)
    m = 4 * 200 * 3 * math.log(200)
    om = sample.sample(na2, nb2, m, seed=77)
    qhat = np.minimum(1, sample.probabilities(na2, nb2, m))
    mu, sd = qhat.sum(), math.sqrt((qhat * (1 - qhat)).sum())
    assert abs(om.nnz - mu) < 5 * sd
    assert om.nnz < m                       # clamping makes E|Omega| < m
    assert np.array_equal(om.qhat, qhat[om.rows, om.cols])
    assert np.allclose(om.w * om.qhat, 1.0, rtol=1e-15)
    key = om.rows * 150 + om.cols
    assert np.all(np.diff(key) > 0)         # row-major order, no duplicates


def test_split_subsets_are_uniform():
    A, B = _mats(d=100, n1=120, n2=130)
    na2, nb2 = (A * A).sum(0), (B * B).sum(0)
    om = sample.sample(na2, nb2, 1e9, seed=8, T=3, split=True)   # everything sampled
    assert om.nnz == 120 * 130
    counts = np.bincount(om.subset, minlength=7)
    assert counts.size == 7
    assert scipy.stats.chisquare(counts).pvalue > 1e-4


def test_zero_norm_rows_never_sampled_from_own_term():
    na2 = np.array([0.0, 1.0, 3.0])
    nb2 = np.array([0.0, 0.0])
    om = sample.sample(na2, nb2, 2.0, seed=1)
    assert not np.any(om.rows == 0)


# ---------------------------------------------------------------- estimator

def test_a_equals_b_diagonal_is_exact():
    """Eq. (2) with A = B: cos = 1 on the diagonal, so M~_ii = ||A_i||^2."""
    A, _ = _mats(d=400, n1=30)
    At, _, na2, _ = sketch.sketch(A, None, seed=3, k=7)
    idx = np.arange(30)
    mt = estimate.estimate(At, At, na2, na2, idx, idx)
    assert np.allclose(mt, na2, rtol=4 * np.finfo(float).eps)


def test_compact_form_equals_entrywise():
    """Appendix B: M~ = D_A A~^T B~ D_B."""
    A, B = _mats()
    At, Bt, na2, nb2 = sketch.sketch(A, B, seed=3, k=9)
    r, c = np.meshgrid(np.arange(A.shape[1]), np.arange(B.shape[1]), indexing="ij")
    mt = estimate.estimate(At, Bt, na2, nb2, r.ravel(), c.ravel()).reshape(r.shape)
    assert np.allclose(mt, estimate.estimate_dense(At, Bt, na2, nb2), rtol=1e-12, atol=1e-14)


def test_orthonormal_pi_gives_exact_product():
    A, B = _mats(d=50)
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((50, 50)))
    At, Bt, na2, nb2 = sketch.sketch_with_pi(Q, A, B)
    r, c = np.meshgrid(np.arange(A.shape[1]), np.arange(B.shape[1]), indexing="ij")
    mt = estimate.estimate(At, Bt, na2, nb2, r.ravel(), c.ravel()).reshape(r.shape)
    assert np.allclose(mt, A.T @ B, atol=1e-12 * np.abs(A.T @ B).max())


def test_estimate_bounded_by_norms_and_zero_norm():
    A, B = _mats()
    A[:, 3] = 0.0
    At, Bt, na2, nb2 = sketch.sketch(A, B, seed=4, k=5)
    r, c = np.meshgrid(np.arange(A.shape[1]), np.arange(B.shape[1]), indexing="ij")
    mt = estimate.estimate(At, Bt, na2, nb2, r.ravel(), c.ravel()).reshape(r.shape)
    bound = np.sqrt(na2)[:, None] * np.sqrt(nb2)[None, :]
    assert np.all(np.abs(mt) <= bound * (1 + 1e-15))
    assert np.all(mt[3] == 0.0)


def test_rescaled_jl_beats_jl_figure_2a(golden_dir):
    """Figure 2(a): for unit vectors (d = 1000, Pi 10 x 1000) the rescaled-JL
    estimate has smaller mean squared error than the plain JL estimate. With the
    cosine uniform on [-1, 1] the plain-JL MSE is (1 + 1/3)/k = 0.133 in closed
    form, next to the printed 0.129; the printed rescaled value is 0.053."""
    import json, os
    gold = json.load(open(os.path.join(golden_dir, "paper_values.json")))["fig2a_mse"]
    d, k, npairs = gold["d"], gold["k"], 1500
    rng = np.random.default_rng(11)
    x = rng.standard_normal((d, npairs))
    x /= np.linalg.norm(x, axis=0)
    t = rng.standard_normal((d, npairs))
    t -= (t * x).sum(0) * x
    t /= np.linalg.norm(t, axis=0)
    cos = rng.uniform(-1, 1, npairs)
    y = cos * x + np.sqrt(1 - cos**2) * t
    P = sketch.pi_block(2024, k, 0, d)
    xs, ys = P @ x, P @ y
    jl = (xs * ys).sum(0)
    resc = estimate.estimate(xs, ys, np.ones(npairs), np.ones(npairs), np.arange(npairs), np.arange(npairs))
    mse_jl = np.mean((jl - cos) ** 2)
    mse_rs = np.mean((resc - cos) ** 2)
    assert abs(mse_jl - (1 + 1 / 3) / k) < 0.25 * (1 + 1 / 3) / k
    assert abs(mse_jl - gold["jl"]) < 0.03
    assert mse_rs < 0.6 * mse_jl
    assert abs(mse_rs - gold["rescaled_jl"]) < 0.025


def test_lemma_b4_entrywise_bound_statistically():
    """Lemma B.4: |M~_ij - A_i^T B_j| <= eps ||A_i|| ||B_j|| with eps ~ sqrt(log(n)/k):
    with k = 400 the worst normalised entry error stays below 7 sqrt(log(2n)/k)."""
    A, B = _mats(d=2000, n1=40, n2=40)
    At, Bt, na2, nb2 = sketch.sketch(A, B, seed=6, k=400)
    r, c = np.meshgrid(np.arange(40), np.arange(40), indexing="ij")
    mt = estimate.estimate(At, Bt, na2, nb2, r.ravel(), c.ravel()).reshape(40, 40)
    err = np.abs(mt - A.T @ B) / (np.sqrt(na2)[:, None] * np.sqrt(nb2)[None, :])
    assert err.max() < 7 * math.sqrt(math.log(80) / 400)

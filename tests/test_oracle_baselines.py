"""Pins of the comparison methods in the oracle (oracle.baselines), against
what the paper and the mathematics fix:

  * SVD(A~^T B~) with Pi = I (k = d) is the best rank-r approximation of
    A^T B: its error is sigma_{r+1}/sigma_1 (Eckart-Young);
  * LELA with every entry sampled (q^ = 1, w = 1) completes the exact A^T B,
    so its error reaches sigma_{r+1}/sigma_1 as well; its first pass is the
    column norms;
  * on the paper's synthetic family (A, B = G D, D_ii = 1/i, Section 4)
    LELA's error lies between the optimum and SMP-PCA's with the same sample
    (Table 1's ordering "Optimal <= LELA <= SMP-PCA"; it has the exact entries
    SMP-PCA estimates), and SMP-PCA's error falls towards LELA's as k grows;
  * for columns from a narrow cone, SMP-PCA is far below SVD(A~^T B~)
    (Figures 2(b), 4(b)).
"""

import numpy as np

import smp_inputs
from oracle import baselines, evaluate, sample, solve


def test_svd_of_sketches_with_identity_pi_is_eckart_young():
    A, B = smp_inputs.gd_pair(300, 60, 50, seed=3)
    A, B = A.numpy().astype(np.float64), B.numpy().astype(np.float64)
    U, s, V = baselines.svd_of_sketches(A, B, 4)          # Pi = I: the sketches are A and B
    M = evaluate.product(A, B)
    assert np.allclose(U.T @ U, np.eye(4), atol=1e-12) and np.allclose(V.T @ V, np.eye(4), atol=1e-12)
    e = evaluate.relative_error(M, U, s, V)
    assert abs(e - evaluate.optimal_error(M, 4)) <= 1e-10


def test_column_norms_are_the_squared_norms():
    A = np.random.default_rng(0).standard_normal((40000, 7))
    got = baselines.column_norms2(A)
    assert np.allclose(got, np.sum(A * A, axis=0), rtol=1e-12)   # and over several 16,384-row chunks


def test_lela_full_observation_reaches_optimum():
    A, B = smp_inputs.gd_pair(400, 50, 40, seed=4)
    A, B = A.numpy(), B.numpy()
    res = baselines.lela(A, B, 3, 1e12, 15, seed=9)
    assert res["omega"].nnz == 50 * 40 and np.all(res["omega"].w == 1.0)
    M = evaluate.product(A, B)
    assert np.allclose(res["mt"], M.ravel(), rtol=1e-14)
    e = evaluate.relative_error(M, res["Uc"], res["sigma"], res["Vc"])
    assert abs(e - evaluate.optimal_error(M, 3)) <= 1e-6 * e


def test_lela_samples_with_the_smp_pca_coins():
    """LELA's first pass and sample are those of Alg. 1 with exact norms:
    the sampled set equals oracle.sample on the column norms."""
    A, B = smp_inputs.gd_pair(500, 80, 70, seed=6)
    A, B = A.numpy(), B.numpy()
    m = solve.default_m(80, 70, 3)
    res = baselines.lela(A, B, 3, m, 5, seed=12)
    ref = sample.sample(np.sum(A.astype(np.float64) ** 2, 0), np.sum(B.astype(np.float64) ** 2, 0), m, 12)
    assert np.array_equal(res["omega"].rows, ref.rows) and np.array_equal(res["omega"].cols, ref.cols)


def test_table1_ordering_on_the_synthetic_family():
    """Optimal <= LELA <= SMP-PCA on A, B = G D (Section 4's synthetic data),
    averaged over seeds; the SMP-PCA error falls towards LELA's with k."""
    d, n, r = 4000, 150, 5
    A, B = smp_inputs.gd_pair(d, n, n, seed=21)
    A, B = A.numpy(), B.numpy()
    M = evaluate.product(A, B)
    e_opt = evaluate.optimal_error(M, r)
    m = solve.default_m(n, n, r)
    e_lela, e_smp = [], {80: [], 640: []}
    for s in range(3):
        res = baselines.lela(A, B, r, m, 10, seed=50 + s)
        e_lela.append(evaluate.relative_error(M, res["Uc"], res["sigma"], res["Vc"]))
        for k in e_smp:
            out = solve.smp_pca(A, B, r, k, m, 10, seed=50 + s)
            e_smp[k].append(evaluate.relative_error(M, out["Uc"], out["sigma"], out["Vc"]))
    lela_mean = np.mean(e_lela)
    assert e_opt <= min(e_lela)
    assert lela_mean <= np.mean(e_smp[640]) < np.mean(e_smp[80])
    assert np.mean(e_smp[640]) - lela_mean < np.mean(e_smp[80]) - lela_mean


def test_smp_pca_beats_svd_of_sketch_product_on_cone():
    A, B = smp_inputs.cone_pair(500, 100, 0.3, 7)
    A, B = A.numpy(), B.numpy()
    M = evaluate.product(A, B)
    res = solve.smp_pca(A, B, 2, 20, 1e9, 10, seed=5)       # every entry sampled
    e_smp = evaluate.relative_error(M, res["Uc"], res["sigma"], res["Vc"])
    U, s, V = baselines.svd_of_sketch_product(A, B, 2, 20, seed=5)
    e_svd = evaluate.relative_error(M, U, s, V)
    assert e_smp < 0.5 * e_svd

"""Pins of the entry-wise sketch in the oracle (oracle.sparse) against what the
definition and the mathematics fix, not against its own formula:

  * Pi times a scipy.sparse matrix built from the same triples (an independent
    sparse product) and the oracle's dense pass on the densified matrix agree
    with it;
  * the order of the triples does not matter, and the sketches of two disjoint
    sets of triples add up to the sketch of their union (the pass is linear);
  * one triple per column gives v Pi[:, l] itself;
  * the BF16 and SRHT forms equal the dense definitions of those sketches;
  * E ||Pi x||^2 = ||x||^2 over seeds (the JL property of the Gaussian Pi);
  * repeated pairs and indices out of range are rejected;
  * the sparse input generator gives each pair once, positive integer counts
    and a power-law column degree.
"""

import numpy as np
import pytest
import scipy.sparse

from oracle import sketch, sparse, srht
from smp_inputs import sparse as spin


def random_entries(rng, d, n, nnz):
    key = rng.choice(d * n, size=nnz, replace=False)
    return (key // n).astype(np.int64), (key % n).astype(np.int32), rng.standard_normal(nnz).astype(np.float32)


def test_matches_scipy_sparse_product():
    rng = np.random.default_rng(1)
    d, n, k = 300, 20, 16
    e = random_entries(rng, d, n, 900)
    Xt, nx2 = sparse.sketch_entries(*e, d, n, seed=5, k=k)
    P = sketch.pi_block(5, k, 0, d)
    S = scipy.sparse.coo_matrix((e[2].astype(np.float64), (e[0], e[1])), shape=(d, n)).tocsc()
    ref = (S.T @ P.T).T
    assert np.allclose(Xt, ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(nx2, np.asarray(S.multiply(S).sum(axis=0)).ravel(), rtol=1e-14)


def test_matches_dense_pass_on_the_bag_of_words_case():
    c = spin.SPARSE_CONFIGS["s1_small"]
    A, B = spin.sparse_pair(c, 11)
    d, n1, n2, k = c["d"], c["n1"], c["n2"], c["k"]
    At, Bt, na2, nb2 = sparse.sketch_pair(A, B, d, n1, n2, 3, k)
    Ad, Bd = spin.densify(A, d, n1), spin.densify(B, d, n2)
    rA, rB, ra, rb = sketch.sketch(Ad, Bd, 3, k)
    for got, ref in ((At, rA), (Bt, rB), (na2, ra), (nb2, rb)):
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-9 * np.abs(ref).max())


def test_order_does_not_matter_and_pushes_add_up():
    rng = np.random.default_rng(2)
    d, n, k = 500, 30, 24
    e = random_entries(rng, d, n, 2000)
    X, nx = sparse.sketch_entries(*e, d, n, 9, k)
    p = rng.permutation(len(e[0]))
    Xp, nxp = sparse.sketch_entries(*(a[p] for a in e), d, n, 9, k)
    assert np.allclose(Xp, X, rtol=1e-12, atol=1e-12) and np.allclose(nxp, nx, rtol=1e-13)
    h = len(e[0]) // 3
    X1, n1 = sparse.sketch_entries(*(a[p[:h]] for a in e), d, n, 9, k)
    X2, n2 = sparse.sketch_entries(*(a[p[h:]] for a in e), d, n, 9, k)
    assert np.allclose(X1 + X2, X, rtol=1e-12, atol=1e-12) and np.allclose(n1 + n2, nx, rtol=1e-13)


def test_one_entry_per_column_is_a_column_of_pi():
    d, n, k = 1000, 6, 10
    rows = np.array([0, 999, 17, 512, 3, 640], dtype=np.int64)
    cols = np.arange(n, dtype=np.int32)
    vals = np.array([1.0, -2.0, 0.5, 3.0, -0.25, 7.0], dtype=np.float32)
    Xt, nx2 = sparse.sketch_entries(rows, cols, vals, d, n, 21, k)
    P = sketch.pi_block(21, k, 0, d)
    for i in range(n):
        assert np.allclose(Xt[:, i], vals[i] * P[:, rows[i]], rtol=1e-15, atol=0)
    assert np.array_equal(nx2, vals.astype(np.float64) ** 2)


def test_bf16_form_equals_the_dense_bf16_definition():
    c = spin.SPARSE_CONFIGS["s1_small"]
    A, B = spin.sparse_pair(c, 12)
    d, n1, n2, k = c["d"], c["n1"], c["n2"], c["k"]
    # non-integer values, so that the rounding of the data matters too
    A = (A[0], A[1], (A[2] * np.float32(1.37)).astype(np.float32))
    At, Bt, na2, nb2 = sparse.sketch_pair(A, B, d, n1, n2, 4, k, fmt="bf16")
    rA, rB, ra, rb = sketch.sketch_lowp(spin.densify(A, d, n1), spin.densify(B, d, n2), 4, k, "bf16")
    for got, ref in ((At, rA), (Bt, rB), (na2, ra), (nb2, rb)):
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-9 * np.abs(ref).max())


def test_srht_form_equals_the_dense_srht():
    rng = np.random.default_rng(3)
    d, n, k = 700, 25, 48     # d not a power of two
    e = random_entries(rng, d, n, 3000)
    Xt, nx2 = sparse.sketch_entries(*e, d, n, 13, k, kind="srht")
    ref, _, rn, _ = srht.sketch(spin.densify(e, d, n), None, 13, k)
    assert np.allclose(Xt, ref, rtol=1e-12, atol=1e-12) and np.allclose(nx2, rn, rtol=1e-13)


def test_squared_norm_unbiased_over_seeds():
    rng = np.random.default_rng(4)
    d, n, k = 2000, 1, 16
    rows = rng.choice(d, 50, replace=False).astype(np.int64)
    vals = rng.standard_normal(50).astype(np.float32)
    cols = np.zeros(50, dtype=np.int32)
    x2 = float(np.sum(vals.astype(np.float64) ** 2))
    est = np.array([np.sum(sparse.sketch_entries(rows, cols, vals, d, n, s, k)[0] ** 2) for s in range(400)])
    # ||Pi x||^2 k / ||x||^2 is chi-square with k degrees of freedom: mean ||x||^2, variance 2 ||x||^4 / k
    assert abs(est.mean() - x2) < 5 * x2 * np.sqrt(2.0 / k / est.size)
    assert abs(est.var() / x2 ** 2 - 2.0 / k) < 0.5 * 2.0 / k


def test_rejects_repeated_pairs_and_bad_indices():
    rows = np.array([1, 2, 1], dtype=np.int64)
    cols = np.array([0, 0, 0], dtype=np.int32)
    vals = np.ones(3, dtype=np.float32)
    with pytest.raises(ValueError, match="more than once"):
        sparse.sketch_entries(rows, cols, vals, 10, 2, 1, 4)
    with pytest.raises(ValueError, match="row index"):
        sparse.sketch_entries(np.array([10]), np.array([0]), np.array([1.0]), 10, 2, 1, 4)
    with pytest.raises(ValueError, match="column index"):
        sparse.sketch_entries(np.array([0]), np.array([2]), np.array([1.0]), 10, 2, 1, 4)
    Xt, nx2 = sparse.sketch_entries(np.zeros(0), np.zeros(0), np.zeros(0), 10, 2, 1, 4)
    assert not Xt.any() and not nx2.any()


def test_generator_pairs_once_counts_and_degrees():
    c = spin.SPARSE_CONFIGS["s1_small"]
    A, B = spin.sparse_pair(c, 5)
    A2, _ = spin.sparse_pair(c, 5)
    assert all(np.array_equal(x, y) for x, y in zip(A, A2))          # seeded
    for (rows, cols, vals), n in ((A, c["n1"]), (B, c["n2"])):
        assert rows.min() >= 0 and rows.max() < c["d"] and cols.min() >= 0 and cols.max() < n
        assert np.unique(cols.astype(np.int64) * c["d"] + rows).size == rows.size
        assert np.all(vals >= 1) and np.all(vals == np.round(vals))
        deg = np.bincount(rows, minlength=c["d"])            # word frequencies: heavy head, long tail
        assert deg.max() > 8 * np.median(deg[deg > 0])
    assert not np.all(np.diff(A[1]) >= 0)                    # arrival order is shuffled

"""Pins of the row-wise multinomial sampler of Appendix D ("Sampling") in the
oracle (oracle.multinomial), against what the appendix and the mathematics
fix rather than against the code itself:

  * the exact 128-bit product behind each draw's target (Python integers);
  * the binary search against a brute-force CDF built entry by entry;
  * m_i equals the appendix's closed form m (||A_i||^2/(2||A||_F^2) + 1/(2 n1))
    and sums to m (Eq. (1) summed over the grid);
  * the row counts are the randomised rounding of m_i;
  * over many seeds the mean multiplicity of (i, j) is q_ij of Eq. (1)
    (unbiased draws), the mean of w_ij 1{(i,j) in Omega} is 1 (so R_Omega is
    unbiased, as with the binomial coins of Alg. 1 step 3), and an entry with
    q_ij = 0 is never drawn;
  * end to end, the multinomial sample gives an error close to the binomial
    one (Appendix D: within a factor of 2).
"""

import numpy as np
import pytest

from oracle import evaluate, multinomial as mn, sample as osa, solve as oso
import smp_inputs


def test_mulhi64_exact_against_python_integers():
    rng = np.random.default_rng(1)
    u = rng.integers(0, 2**63, size=2000, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=2000).astype(np.uint64)
    t = rng.integers(0, 2**53, size=2000, dtype=np.int64).astype(np.uint64)
    edge_u = np.array([0, 1, 2**64 - 1, 2**63, 2**32 - 1, 2**32], dtype=np.uint64)
    edge_t = np.array([2**53 - 1, 1, 2**53 - 1, 2**52, 2**53 - 1, 0], dtype=np.uint64)
    u = np.concatenate([u, edge_u])
    t = np.concatenate([t, edge_t])
    got = mn.mulhi64(u, t)
    want = [(int(a) * int(b)) >> 64 for a, b in zip(u, t)]
    assert [int(x) for x in got] == want


def test_locate_matches_brute_force_cdf():
    rng = np.random.default_rng(2)
    for n2 in (1, 2, 7, 64, 333):
        b = rng.integers(0, 1000, size=n2).astype(np.uint64)
        b[rng.random(n2) < 0.2] = 0                         # zero-weight columns
        bcum = np.cumsum(b, dtype=np.uint64)
        for a_row in (0, 3, 997):
            w = np.uint64(a_row) + b                          # the row's weights, entry by entry
            if int(w.sum()) == 0:
                continue
            cdf = np.cumsum(w, dtype=np.uint64)
            t = rng.integers(0, int(cdf[-1]), size=500).astype(np.uint64)
            t[:2] = [0, int(cdf[-1]) - 1]
            got = mn.locate(t, np.full(t.shape, a_row, dtype=np.uint64), bcum)
            want = np.searchsorted(cdf, t, side="right")
            assert np.array_equal(got, want)
            assert np.all(w[got] > 0)                          # never a zero-weight column


def _norms(n1, n2, seed=0, heavy=False):
    rng = np.random.default_rng(seed)
    na2 = (rng.random(n1) ** 3 * 10).astype(np.float32).astype(np.float64)
    nb2 = (rng.random(n2) ** 3 * 10).astype(np.float32).astype(np.float64)
    if heavy:
        nb2[0] = 1e3
    return na2, nb2


@pytest.mark.parametrize("n1,n2,m", [(40, 30, 500.0), (200, 17, 3000.5), (5, 300, 80.0)])
def test_row_expectations_follow_appendix_d(n1, n2, m):
    na2, nb2 = _norms(n1, n2)
    a, b, bcum, total, FA, FB = mn.integer_weights(na2, nb2)
    counts, mi = mn.row_counts(total, m, seed=7)
    closed = m * (na2 / (2.0 * na2.sum()) + 1.0 / (2.0 * n1))      # the appendix's m_i
    assert np.allclose(mi, closed, rtol=1e-9, atol=1e-12 * m)
    assert abs(mi.sum() - m) <= 1e-9 * m
    assert np.all((counts == np.floor(mi)) | (counts == np.floor(mi) + 1))
    # q_ij of Eq. (1), summed over the row, is m_i
    q = osa.probabilities(na2, nb2, m)
    assert np.allclose(q.sum(axis=1), mi, rtol=1e-9)


def test_draw_frequencies_and_unbiased_weights_over_seeds():
    n1, n2, m = 4, 6, 30.0
    na2, nb2 = _norms(n1, n2, seed=3, heavy=True)
    na2[2] = 0.0                                                   # q_23 = 0: (2, 3) must never be drawn
    nb2[3] = 0.0
    q = osa.probabilities(na2, nb2, m)
    S = 3000
    mult = np.zeros((n1, n2))
    wsum = np.zeros((n1, n2))
    counts = np.zeros(n1)
    for s in range(S):
        om = mn.sample(na2, nb2, m, seed=1000 + s)
        np.add.at(mult, (om.rows, om.cols), om.count)
        np.add.at(wsum, (om.rows, om.cols), om.w)
        counts += om.row_draws
        assert np.array_equal(np.bincount(om.rows, weights=om.count, minlength=n1).astype(np.int64), om.row_draws)
        assert np.all(np.diff(om.rows * n2 + om.cols) > 0)       # row-major, each entry once
    mean, var_bound = mult / S, q / S                              # multiplicities: variance <= q (c fixed) + rounding
    z = np.abs(mean - q) / np.sqrt(np.maximum(var_bound * 1.5, 1e-12))
    assert np.all(z < 5.0), z.max()
    assert q[2, 3] == 0.0 and mult[2, 3] == 0
    ok = q > 0
    assert np.all(np.abs(wsum[ok] / S - 1.0) < 5.0 * np.sqrt(1.5 / (q[ok] * S)) + 1e-12)
    mi = q.sum(axis=1)
    assert np.all(np.abs(counts / S - mi) < 5.0 * np.sqrt(0.25 / S) + 1e-9)


def test_zero_norms_and_tiny_m():
    na2 = np.zeros(5)
    nb2 = np.zeros(4)
    om = mn.sample(na2, nb2, 10.0, seed=1)
    assert om.nnz == 0
    na2, nb2 = _norms(6, 5)
    om = mn.sample(na2, nb2, 1e-3, seed=2)                          # m_i < 1: most rows draw nothing
    assert om.row_draws.sum() <= 6


def test_end_to_end_error_close_to_binomial():
    """Appendix D: the multinomial model's error is within a factor of 2 of
    the binomial model's. On the small workload (d = 2,000, n = 200, k = 50,
    r = 5) both samplers feed the same sketches into WAltMin."""
    c = smp_inputs.CONFIGS["c1_small"]
    A, B = smp_inputs.latent_pair(c["d"], c["n1"], c["n2"], c["R"], c["sigma"], c["alpha"], smp_inputs.SEED_BASE)
    A, B = A.numpy(), B.numpy()
    m = oso.default_m(c["n1"], c["n2"], c["r"])
    M = evaluate.product(A, B)
    errs = {}
    for sampler in ("binomial", "multinomial"):
        res = oso.smp_pca(A, B, c["r"], c["k"], m, c["T"], smp_inputs.SEED_BASE, sampler=sampler)
        errs[sampler] = evaluate.relative_error(M, res["Uc"], res["sigma"], res["Vc"])
    assert errs["multinomial"] <= 2.0 * errs["binomial"]
    assert errs["binomial"] <= 2.0 * errs["multinomial"]

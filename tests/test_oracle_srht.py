"""Pins of the SRHT sketch in the oracle (oracle.srht) against what the
transform's definition and the mathematics fix:

  * the +-1 pattern (-1)^popcount(rho & l) is Sylvester's Hadamard matrix
    (scipy.linalg.hadamard, an independent construction);
  * rows of Pi for distinct rho are orthogonal with squared norm D/k, and
    E[Pi^T Pi] = I: averaged over seeds, A~^T B~ tends to A^T B with the
    spread the JL variance allows;
  * the signs are balanced and the rows uniform over [0, D);
  * end to end, SMP-PCA with the SRHT sketch reaches an error close to the
    Gaussian sketch's (Section 4 footnote: the same quality of the output).
"""

import numpy as np
import scipy.linalg

import smp_inputs
from oracle import evaluate, solve, srht


def test_hadamard_pattern_is_sylvester():
    for D in (1, 2, 8, 64, 256):
        H = scipy.linalg.hadamard(D)
        got = srht.hadamard_signs(np.arange(D), np.arange(D))
        assert np.array_equal(got, H.astype(np.float64))


def test_padded_size():
    assert [srht.padded_size(d) for d in (1, 2, 3, 1000, 1024, 1025, 200_000)] == [1, 2, 4, 1024, 1024, 2048, 262_144]


def test_rows_orthogonal_and_scaled():
    d = D = 256
    k = 40
    P = srht.pi_block(7, k, d, 0, d)
    rho = srht.rows(7, k, D)
    G = P @ P.T
    same = rho[:, None] == rho[None, :]
    assert np.allclose(G[same], D / k) and np.allclose(G[~same], 0.0, atol=1e-12)
    assert np.all(np.abs(P) == 1.0 / np.sqrt(k))


def test_signs_balanced_rows_uniform():
    s = srht.signs(3, 0, 200_000)
    assert abs(s.mean()) < 5.0 / np.sqrt(200_000)
    rho = srht.rows(3, 64_000, 64)
    counts = np.bincount(rho, minlength=64)
    chi2 = ((counts - 1000.0) ** 2 / 1000.0).sum()
    assert chi2 < 63 + 5 * np.sqrt(2 * 63)


def test_unbiased_inner_products():
    """E[Pi^T Pi] = I: mean of A~^T B~ over seeds -> A^T B."""
    d, n, k = 300, 6, 16
    rng = np.random.default_rng(0)
    A = rng.standard_normal((d, n))
    B = rng.standard_normal((d, n))
    M = A.T @ B
    S = 400
    acc = np.zeros((n, n))
    sq = np.zeros((n, n))
    for s in range(S):
        At, Bt, na2, nb2 = srht.sketch(A, B, 100 + s, k)
        X = At.T @ Bt
        acc += X
        sq += X * X
    mean = acc / S
    sd = np.sqrt(np.maximum(sq / S - mean ** 2, 1e-12) / S)
    assert np.all(np.abs(mean - M) < 5 * sd)
    assert np.allclose(na2, (A * A).sum(0)) and np.allclose(nb2, (B * B).sum(0))


def test_end_to_end_error_close_to_gaussian():
    c = smp_inputs.CONFIGS["c1_small"]
    A, B = smp_inputs.latent_pair(c["d"], c["n1"], c["n2"], c["R"], c["sigma"], c["alpha"], smp_inputs.SEED_BASE)
    A, B = A.numpy(), B.numpy()
    m = solve.default_m(c["n1"], c["n2"], c["r"])
    M = evaluate.product(A, B)
    e = {}
    for kind in ("gaussian", "srht"):
        res = solve.smp_pca(A, B, c["r"], c["k"], m, c["T"], smp_inputs.SEED_BASE, sketch_kind=kind)
        e[kind] = evaluate.relative_error(M, res["Uc"], res["sigma"], res["Vc"])
    assert e["srht"] <= 1.5 * e["gaussian"] and e["gaussian"] <= 1.5 * e["srht"]

"""Pins for the oracle's random streams: Philox4x32-10 against rocRAND's
independent implementation (black box), and the Gaussian transform against
the normal distribution and the closed-form variance of the JL estimator."""

import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

from oracle import philox, gaussian, sketch


@pytest.fixture(scope="module")
def kat_binary(golden_dir, tmp_path_factory):
    src = os.path.join(golden_dir, "philox_kat.cpp")
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include/rocrand"):
        pytest.skip("g++ or rocRAND headers not available")
    out = str(tmp_path_factory.mktemp("kat") / "philox_kat")
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", src, "-o", out],
                   check=True, capture_output=True)
    return out


def test_philox_matches_rocrand(kat_binary):
    rng = np.random.default_rng(7)
    n = 3000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    # edge words: all-zero, all-ones, and the counter layout actually used
    ctr[:4] = [[0, 0, 0, 0], [2**32 - 1] * 4, [5, 123456, philox.TAG_PI, 0], [0, 7, philox.TAG_SAMPLE, 1]]
    key[:4] = [[0, 0], [2**32 - 1] * 2, [161006656, 0], [2**32 - 1, 3]]
    lines = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, key))
    res = subprocess.run([kat_binary], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(t) for t in ln.split()] for ln in res.stdout.strip().splitlines()], dtype=np.uint64)
    ours = np.empty_like(ref)
    for i in range(n):
        out = philox.philox4x32_10(ctr[i, 0], ctr[i, 1], ctr[i, 2], ctr[i, 3], int(key[i, 0]), int(key[i, 1]))
        ours[i] = [int(o) for o in out]
    assert np.array_equal(ours, ref)


def test_philox_vectorised_equals_scalar():
    rows = np.arange(0, 40, dtype=np.int64)[:, None] * 977 + (1 << 33)
    cb = np.arange(0, 6, dtype=np.int64)[None, :]
    w = philox.stream_words(99, philox.TAG_PI, rows, cb)
    k0, k1 = philox.seed_key(99)
    for r in range(0, 40, 13):
        for c in range(6):
            l = int(rows[r, 0])
            s = philox.philox4x32_10(c, l & 0xFFFFFFFF, philox.TAG_PI, l >> 32, k0, k1)
            assert all(int(w[q][r, c]) == int(s[q]) for q in range(4))


def test_uniforms_range_and_exactness():
    a = np.array([0, 255, 256, 2**32 - 1], dtype=np.uint32)
    u, phi = gaussian.uniforms(a, a)
    assert u[0] == 2.0**-24 and u[1] == 2.0**-24 and u[2] == 2 * 2.0**-24 and u[3] == 1.0
    assert phi[0] == 0.0 and phi[3] == 1.0 - 2.0**-24
    assert np.all(np.float32(u) == u)       # exact in FP32 too


def test_gaussian_distribution():
    z = sketch.gaussian_block(12345, 64, 0, 4096).ravel()       # 262144 variates
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(scipy.stats.kurtosis(z, fisher=False) - 3.0) < 5 * np.sqrt(24.0 / n)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    # the lanes of one call and neighbouring rows are uncorrelated
    Z = sketch.gaussian_block(12345, 64, 0, 4096)
    C = np.corrcoef(Z)
    off = C[~np.eye(64, dtype=bool)]
    assert np.max(np.abs(off)) < 6 / np.sqrt(4096)


def test_pi_variance_is_one_over_k():
    for k in (10, 50, 400):
        P = sketch.pi_block(3, k, 1000, 1000 + 20000 // k * 10)
        v = P.var()
        assert abs(v * k - 1.0) < 6 * np.sqrt(2.0 / P.size)


def test_jl_inner_product_variance_closed_form():
    """For Pi with i.i.d. N(0, 1/k) entries, Var(<Pi x, Pi y>) = (|x|^2|y|^2 + <x,y>^2)/k.
    Checked for unit x, y at three angles over many independent Pi (seeds)."""
    d, k, trials = 200, 10, 600
    rng = np.random.default_rng(1)
    x = rng.standard_normal(d)
    x /= np.linalg.norm(x)
    t = rng.standard_normal(d)
    t -= t.dot(x) * x
    t /= np.linalg.norm(t)
    for cos in (0.0, 0.6, 0.95):
        y = cos * x + np.sqrt(1 - cos**2) * t
        est = np.empty(trials)
        for s in range(trials):
            P = sketch.pi_block(1000 + s, k, 0, d)
            est[s] = (P @ x).dot(P @ y)
        var_th = (1 + cos**2) / k
        assert abs(est.mean() - cos) < 5 * np.sqrt(var_th / trials)
        assert abs(est.var() / var_th - 1) < 5 * np.sqrt(2.0 / trials)

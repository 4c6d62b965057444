"""Pins for the oracle's narrow-format rounding and the low-precision sketch
(Alg. 1 step 2 with the GEMM operands rounded; the paper fixes no precision).

* round_bf16 against torch's float32 -> bfloat16 conversion (an independent
  library implementation of round-to-nearest-even) and hand-computed ties.
* sketch_lowp against the FP64 sketch through the deterministic rounding
  bound |R(z) R(x) - z x| <= (2u + u^2) |z x| (u = 2^-8, the unit roundoff of
  an 8-significant-bit format), and against an exact case.
"""

import numpy as np
import torch

from oracle import rounding, sketch


def test_round_bf16_matches_torch_over_the_fp32_range():
    rng = np.random.default_rng(0)
    mant = rng.standard_normal(200000)
    expo = rng.uniform(-140, 128, 200000)
    with np.errstate(over="ignore"):
        x = (mant * np.exp2(expo)).astype(np.float32)
    x = np.concatenate([x, np.float32([0.0, -0.0, 1e-45, -1e-45, 3.4028235e38, -3.4028235e38,
                                       1.1754944e-38, 9.2e-41])])
    x = x[np.isfinite(x)].astype(np.float64)
    ours = rounding.round_bf16(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_round_bf16_ties_go_to_even():
    u = 2.0 ** -7    # spacing of bfloat16 in [1, 2)
    cases = {
        1.0 + u / 2: 1.0,                # tie between 1 (even) and 1 + u (odd)
        1.0 + 3 * u / 2: 1.0 + 2 * u,    # tie between 1 + u (odd) and 1 + 2u (even)
        1.0 + u / 2 + 2.0 ** -30: 1.0 + u,
        -(1.0 + u / 2): -1.0,
        3.0: 3.0,
        2.0 ** -133: 2.0 ** -133,        # smallest subnormal
        2.0 ** -134: 0.0,                # half of it: tie to even (zero)
        3 * 2.0 ** -134: 2.0 ** -132,    # 1.5 subnormal steps: tie to the even step 2
    }
    x = np.array(list(cases.keys()))
    assert np.array_equal(rounding.round_bf16(x), np.array(list(cases.values())))
    assert np.isinf(rounding.round_bf16(np.array([rounding.BF16_MAX * (1 + 2.0 ** -8)]))[0])
    assert rounding.round_bf16(np.array([rounding.BF16_MAX * (1 + 2.0 ** -9)]))[0] == rounding.BF16_MAX


def _data(d, n, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((d, n)) * (np.arange(1, n + 1) ** -0.5)).astype(np.float32).astype(np.float64)


def test_sketch_bf16_within_the_rounding_bound_of_the_exact_sketch():
    d, n1, n2, k, seed = 700, 9, 6, 12, 11
    A, B = _data(d, n1, 1), _data(d, n2, 2)
    At, Bt, na2, nb2 = sketch.sketch_lowp(A, B, seed, k, "bf16", chunk=256)
    Ae, Be, na2e, nb2e = sketch.sketch(A, B, seed, k, chunk=256)
    u = 2.0 ** -8
    Z = np.abs(sketch.gaussian_block(seed, k, 0, d)) / np.sqrt(k)
    for got, exact, X in ((At, Ae, A), (Bt, Be, B)):
        bound = (2 * u + u * u) * (Z @ np.abs(X))
        assert np.all(np.abs(got - exact) <= bound * (1 + 1e-12) + 1e-300)
        # the rounding is really applied: errors of the order of u, not zero
        rel = np.linalg.norm(got - exact) / np.linalg.norm(exact)
        assert 1e-2 * u < rel < 2 * u
    assert np.array_equal(na2, na2e) and np.array_equal(nb2, nb2e)


def test_sketch_bf16_of_bf16_exact_data_only_rounds_pi():
    """Small integers are exact in bfloat16, so only Pi is rounded."""
    d, n, k, seed = 300, 5, 8, 4
    rng = np.random.default_rng(5)
    A = rng.integers(-100, 101, size=(d, n)).astype(np.float64)
    At, _, _, _ = sketch.sketch_lowp(A, None, seed, k, "bf16", chunk=128)
    Zr = torch.from_numpy(sketch.gaussian_block(seed, k, 0, d).astype(np.float32)).to(torch.bfloat16)
    ref = Zr.to(torch.float64).numpy() @ A / np.sqrt(k)
    # FP64 Z -> bf16 and FP64 Z -> FP32 -> bf16 differ only where the FP32 step lands on a bf16 tie
    assert np.allclose(At, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_sketch_bf16_a_equals_b_shares_the_result():
    A = _data(200, 7, 3)
    At, Bt, na2, nb2 = sketch.sketch_lowp(A, None, 2, 5, "bf16")
    assert At is Bt and na2 is nb2
    At2, Bt2, _, _ = sketch.sketch_lowp(A, A, 2, 5, "bf16")
    assert np.array_equal(At, At2) and np.array_equal(At2, Bt2)


# ---------------------------------------------------------------- FP8 E4M3 with E8M0 block scales

def test_round_e4m3_matches_torch_in_range():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(200000) * np.exp2(rng.uniform(-14, 9, 200000))
    x = x.astype(np.float32).astype(np.float64)
    x = np.concatenate([x[np.abs(x) <= 448], [0.0, -0.0, 448.0, -448.0, 2.0 ** -9, 2.0 ** -6, 2.0 ** -7 * 1.0625]])
    ours = rounding.round_e4m3(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_round_e4m3_ties_and_subnormals():
    cases = {
        1.0 + 1 / 16: 1.0,          # tie between 1 (even) and 1.125 (odd)
        1.0 + 3 / 16: 1.25,         # tie between 1.125 (odd) and 1.25 (even)
        2.0 ** -9: 2.0 ** -9,       # smallest subnormal
        2.0 ** -10: 0.0,            # half of it: tie to even (zero)
        3 * 2.0 ** -10: 2.0 ** -8,  # 1.5 subnormal steps: tie to the even step 2
        240.0: 240.0,
        232.0: 224.0,               # tie between 224 (even) and 240 (odd)
        -5.3: -5.5,                 # spacing 0.5 in [4, 8)
    }
    x = np.array(list(cases.keys()))
    assert np.array_equal(rounding.round_e4m3(x), np.array(list(cases.values())))


def test_mx_scale_exponent_is_the_smallest_fitting_power_of_two():
    rng = np.random.default_rng(2)
    amax = np.abs(rng.standard_normal(50000)) * np.exp2(rng.uniform(-60, 60, 50000))
    amax = np.concatenate([amax.astype(np.float32).astype(np.float64), 448.0 * np.exp2(np.arange(-20, 21))])
    e = rounding.mx_scale_exponent(amax)
    assert np.all(amax <= 448.0 * np.exp2(e.astype(np.float64)))
    assert np.all(amax > 448.0 * np.exp2(e.astype(np.float64) - 1))
    assert np.array_equal(rounding.mx_scale_exponent(448.0 * np.exp2(np.arange(-20, 21))), np.arange(-20, 21))
    assert rounding.mx_scale_exponent(np.array([0.0]))[0] == 0
    assert rounding.mx_scale_exponent(np.array([1e-300]))[0] == -127      # clamped to the E8M0 range


def test_e4m3_blocks_fit_the_range_and_the_rounding_bound():
    rng = np.random.default_rng(3)
    X = (rng.standard_normal((200, 9)) * np.exp2(rng.uniform(-20, 20, 9))).astype(np.float32).astype(np.float64)
    Q = rounding.quantize_e4m3_blocks(X)
    u = 2.0 ** -4
    for b0 in range(0, 200, 32):
        blk, q = X[b0:b0 + 32], Q[b0:b0 + 32]
        sc = np.exp2(rounding.mx_scale_exponent(np.abs(blk).max(axis=0)).astype(np.float64))
        assert np.all(np.abs(blk / sc) <= 448.0)
        assert np.all(np.abs(q - blk) <= u * np.abs(blk) + 2.0 ** -10 * sc)
        assert np.array_equal(q / sc, rounding.round_e4m3(q / sc))        # representable after scaling


def test_sketch_fp8_within_the_rounding_bound_and_independent_of_chunking():
    d, n, k, seed = 400, 6, 10, 13
    rng = np.random.default_rng(4)
    A = (rng.standard_normal((d, n)) * (np.arange(1, n + 1) ** -0.7)).astype(np.float32).astype(np.float64)
    At, _, na2, _ = sketch.sketch_lowp(A, None, seed, k, "fp8", chunk=64)
    At2, _, _, _ = sketch.sketch_lowp(A, None, seed, k, "fp8", chunk=96)
    assert np.allclose(At, At2, rtol=0, atol=1e-13 * np.abs(At).max())      # blocks follow global rows
    Ae, _, na2e, _ = sketch.sketch(A, None, seed, k)
    assert np.allclose(na2, na2e, rtol=1e-14)
    Z = np.abs(sketch.gaussian_block(seed, k, 0, d))
    u = 2.0 ** -4
    sc = np.empty_like(A)
    for b0 in range(0, d, 32):
        e = rounding.mx_scale_exponent(np.abs(A[b0:b0 + 32]).max(axis=0))
        sc[b0:b0 + 32] = np.exp2(e.astype(np.float64))
    bound = ((2 * u + u * u) * (Z @ np.abs(A)) + (1 + u) * (Z @ (2.0 ** -10 * sc))) / np.sqrt(k)
    assert np.all(np.abs(At - Ae) <= bound * (1 + 1e-12))
    rel = np.linalg.norm(At - Ae) / np.linalg.norm(Ae)
    assert 1e-3 < rel < 0.2

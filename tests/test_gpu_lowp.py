"""GPU parity of the low-precision sketch variants against the oracle's
definitions of them (``sketch_lowp``: the exact product of the rounded
operands): BF16 (operands rounded to bfloat16, FP32 accumulation) and FP8
(E4M3 operands with E8M0 data block scales, FP32 accumulation; tolerance with
the FP8 tests below), and of the solves end to end.

Tolerances (derived from the arithmetic):
  sketch  per column ||dA~_i|| / ||A~_i|| <= 2e-4. The GPU rounds its FP32
          Box-Muller draw (hardware log/sin/cos, a few FP32 ulps from the FP64
          value) to bfloat16, the oracle its FP64 draw. The two roundings differ
          where the draw lies within ~4 ulp_32 of a bfloat16 rounding midpoint:
          probability ~2^-14 per entry, each such entry moving its product by
          one bfloat16 ulp (2^-8 relative). Summed over d rows with random
          signs this is sqrt(2^-14) * 2^-8 ~ 3e-5 of the column norm; FP32
          accumulation adds ~1e-6.
  norms   unrounded FP32 data, compensated sums: relative 1e-6 (as FP32).
  solve   e_gpu within 1e-3 (relative) of the oracle's e with the same
          BF16 definition of the sketch: the sketch differences above move
          the estimates M~_ij by ~1e-4 relative at most.
"""

import numpy as np
import pytest
import torch

import smp_inputs
from conftest import gpu_available
from gpu_common import DEV, SEED, latent, log
from oracle import evaluate as oev
from oracle import gaussian, philox, rounding
from oracle import sketch as osk
from oracle import solve as oso

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL_SKETCH = 2e-4


@pytest.fixture(scope="module")
def api():
    from paper_1610_06656_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def _col_rel(got_t, ref):
    g = got_t.T.astype(np.float64)
    num = np.linalg.norm(g - ref, axis=0)
    den = np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
    return float(np.max(num / den))


def _bf16_params(api, d, n1, n2, k, **kw):
    return api.make_params(d, n1, n2, k, r=1, prec=api.SMP_PREC_BF16, **kw)


def _sketch_gpu(api, ctx, p, Ad, Bd, n1, n2, k):
    At = torch.empty(n1, k, device=DEV)
    Bt = torch.empty(n2, k, device=DEV)
    na2 = torch.empty(n1, device=DEV)
    nb2 = torch.empty(n2, device=DEV)
    ctx.smp_sketch(p, Ad, Bd, At, Bt, na2, nb2)
    torch.cuda.synchronize()
    return At.cpu().numpy(), Bt.cpu().numpy(), na2.cpu().numpy(), nb2.cpu().numpy()


SKETCH_CASES = {
    "c1": dict(d=2000, n1=200, n2=200, k=50),
    "ragged": dict(d=1037, n1=77, n2=131, k=37),
    "k400_tiles": dict(d=20000, n1=300, n2=1100, k=400),
    "k1024_chunks": dict(d=4096, n1=129, n2=64, k=1024),
    "k700_wide_chunks": dict(d=3000, n1=300, n2=77, k=700),
    "k2000_wide_chunks": dict(d=1500, n1=90, n2=41, k=2000),
    "tiny": dict(d=3, n1=1, n2=5, k=1),
    "one_block_tail": dict(d=130, n1=513, n2=2, k=81),
    "even_not_quad": dict(d=3000, n1=258, n2=130, k=400),   # n even, not a multiple of 4: 8-byte row loads
}


@pytest.mark.parametrize("name", list(SKETCH_CASES))
def test_sketch_bf16_parity(api, ctx, name):
    c = SKETCH_CASES[name]
    log(f"bf16 sketch {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=min(5, c["n1"], c["n2"]))
    p = _bf16_params(api, c["d"], c["n1"], c["n2"], c["k"])
    At, Bt, na2, nb2 = _sketch_gpu(api, ctx, p, Ad, Bd, c["n1"], c["n2"], c["k"])
    oAt, oBt, ona2, onb2 = osk.sketch_lowp(A.numpy(), B.numpy(), p.seed, c["k"], "bf16")
    ea, eb = _col_rel(At, oAt), _col_rel(Bt, oBt)
    log(f"  column rel err A {ea:.2e} B {eb:.2e}")
    assert ea < TOL_SKETCH and eb < TOL_SKETCH
    assert np.allclose(na2, ona2, rtol=1e-6, atol=0)
    assert np.allclose(nb2, onb2, rtol=1e-6, atol=0)


@pytest.mark.parametrize("name", ["c1", "ragged", "k1024_chunks", "one_block_tail"])
def test_sketch_bf16_regenerating_pass_parity(api, ctx, name, monkeypatch):
    """The BF16 pass that regenerates Pi inside each workgroup (selected with
    SMP_SKETCH_BF16_STORED=0; the default pass stores Pi once per push) meets
    the same bar against the oracle."""
    monkeypatch.setenv("SMP_SKETCH_BF16_STORED", "0")
    c = SKETCH_CASES[name]
    log(f"bf16 regenerating sketch {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=min(5, c["n1"], c["n2"]))
    p = _bf16_params(api, c["d"], c["n1"], c["n2"], c["k"])
    At, Bt, na2, nb2 = _sketch_gpu(api, ctx, p, Ad, Bd, c["n1"], c["n2"], c["k"])
    oAt, oBt, ona2, onb2 = osk.sketch_lowp(A.numpy(), B.numpy(), p.seed, c["k"], "bf16")
    assert _col_rel(At, oAt) < TOL_SKETCH and _col_rel(Bt, oBt) < TOL_SKETCH
    assert np.allclose(na2, ona2, rtol=1e-6, atol=0)
    assert np.allclose(nb2, onb2, rtol=1e-6, atol=0)


def test_sketch_bf16_scalar_path_zero_column_and_b_is_a(api, ctx):
    d, n1, n2, k = 700, 45, 33, 21
    A, B, _, _ = latent(d, n1, n2)
    A[:, 7] = 0.0
    Afull = torch.zeros(d, n1 + 3)
    Afull[:, :n1] = A
    Ad = Afull.to(DEV)[:, :n1]                 # lda = n1 + 3 (odd): scalar load path
    p = _bf16_params(api, d, n1, n2, k)
    At, Bt, _, _ = _sketch_gpu(api, ctx, p, Ad, B.to(DEV), n1, n2, k)
    oAt, oBt, _, _ = osk.sketch_lowp(A.numpy(), B.numpy(), p.seed, k, "bf16")
    assert np.all(At[7] == 0.0)
    keep = np.arange(n1) != 7
    assert _col_rel(At[keep], oAt[:, keep]) < TOL_SKETCH
    assert _col_rel(Bt, oBt) < TOL_SKETCH
    # B = A (PCA case)
    n = 96
    A2, _, Ad2, _ = latent(1500, n, n, same=True)
    p2 = _bf16_params(api, 1500, n, n, 40, b_is_a=True)
    At2 = torch.empty(n, 40, device=DEV)
    Bt2 = torch.empty(n, 40, device=DEV)
    na = torch.empty(n, device=DEV)
    nb = torch.empty(n, device=DEV)
    ctx.smp_sketch(p2, Ad2, None, At2, Bt2, na, nb)
    torch.cuda.synchronize()
    oAt2, _, _, _ = osk.sketch_lowp(A2.numpy(), None, p2.seed, 40, "bf16")
    assert _col_rel(At2.cpu().numpy(), oAt2) < TOL_SKETCH
    assert torch.equal(At2, Bt2)


def test_sketch_bf16_streaming_push_any_order(api, ctx):
    d, n1, n2, k = 3000, 130, 70, 64
    A, B, Ad, Bd = latent(d, n1, n2)
    p = _bf16_params(api, d, n1, n2, k)
    st = ctx.smp_sketch_begin(p)
    for l0, l1 in [(2000, 3000), (0, 1), (1, 1999), (1999, 2000)]:
        ctx.smp_sketch_push(st, Ad[l0:l1], Bd[l0:l1], l0)
    At = torch.empty(n1, k, device=DEV)
    Bt = torch.empty(n2, k, device=DEV)
    na2 = torch.empty(n1, device=DEV)
    nb2 = torch.empty(n2, device=DEV)
    ctx.smp_sketch_end(st, At, Bt, na2, nb2)
    torch.cuda.synchronize()
    ctx.smp_sketch_free(st)
    oAt, oBt, ona2, _ = osk.sketch_lowp(A.numpy(), B.numpy(), p.seed, k, "bf16")
    assert _col_rel(At.cpu().numpy(), oAt) < TOL_SKETCH
    assert _col_rel(Bt.cpu().numpy(), oBt) < TOL_SKETCH
    assert np.allclose(na2.cpu().numpy(), ona2, rtol=1e-6)


@pytest.mark.parametrize("prec_name", ["bf16", "fp8"])
@pytest.mark.parametrize("name", ["k400_tiles", "ragged"])
def test_sketch_pi_windows(api, ctx, name, prec_name, monkeypatch):
    """The stored-Pi passes draw Pi one bounded window at a time (Alg. 1
    step 2: Pi is drawn, not kept). With a 1 MiB window the k = 400 case runs
    16 BF16 / 8 FP8 windows (the ragged one a single window and a tail); each
    window's launch adds into the partials of the ones before. The result
    meets the oracle's bar and differs from the one-window pass only by the
    FP32 rounding of those additions."""
    c = SKETCH_CASES[name] if prec_name == "bf16" else FP8_CASES[name]
    prec = api.SMP_PREC_BF16 if prec_name == "bf16" else api.SMP_PREC_FP8
    tol = TOL_SKETCH if prec_name == "bf16" else TOL_FP8
    log(f"{prec_name} windowed sketch {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=min(5, c["n1"], c["n2"]))
    oAt, oBt, ona2, onb2 = osk.sketch_lowp(A.numpy(), B.numpy(), SEED, c["k"], prec_name)
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], r=1, prec=prec, seed=SEED)
    outs = []
    for mb in ("1", "4096"):
        monkeypatch.setenv("SMP_PI_WINDOW_MB", mb)
        outs.append(_sketch_gpu(api, ctx, p, Ad, Bd, c["n1"], c["n2"], c["k"]))
    for At, Bt, na2, nb2 in outs:
        assert _col_rel(At, oAt) < tol and _col_rel(Bt, oBt) < tol
        assert np.allclose(na2, ona2, rtol=1e-6, atol=0) and np.allclose(nb2, onb2, rtol=1e-6, atol=0)
    assert _col_rel(outs[0][0], outs[1][0].T.astype(np.float64)) < 1e-6
    assert _col_rel(outs[0][1], outs[1][1].T.astype(np.float64)) < 1e-6


def test_sketch_bf16_streaming_pushes_span_windows(api, ctx, monkeypatch):
    """Streaming pushes larger than one Pi window (1 MiB: 1,280 rows at
    k = 400) and out of order."""
    monkeypatch.setenv("SMP_PI_WINDOW_MB", "1")
    d, n1, n2, k = 9000, 130, 70, 400
    A, B, Ad, Bd = latent(d, n1, n2)
    cx = ctx
    p = _bf16_params(api, d, n1, n2, k, seed=SEED)
    st = cx.smp_sketch_begin(p)
    for l0, l1 in [(5000, 9000), (0, 17), (17, 5000)]:
        cx.smp_sketch_push(st, Ad[l0:l1], Bd[l0:l1], l0)
    At = torch.empty(n1, k, device=DEV)
    Bt = torch.empty(n2, k, device=DEV)
    na2 = torch.empty(n1, device=DEV)
    nb2 = torch.empty(n2, device=DEV)
    cx.smp_sketch_end(st, At, Bt, na2, nb2)
    torch.cuda.synchronize()
    cx.smp_sketch_free(st)
    oAt, oBt, ona2, _ = osk.sketch_lowp(A.numpy(), B.numpy(), p.seed, k, "bf16")
    assert _col_rel(At.cpu().numpy(), oAt) < TOL_SKETCH
    assert _col_rel(Bt.cpu().numpy(), oBt) < TOL_SKETCH
    assert np.allclose(na2.cpu().numpy(), ona2, rtol=1e-6)


def _pi_rows_bf16(seed, k, rows_c, d):
    """R(Z(c, l)) / sqrt(k) for selected sketch rows c and all l < d."""
    out = np.empty((len(rows_c), d))
    ls = np.arange(d, dtype=np.int64)
    for t, c in enumerate(rows_c):
        w = philox.stream_words(seed, philox.TAG_PI, ls, np.full(d, c // 4, dtype=np.int64))
        out[t] = rounding.round_bf16(gaussian.normals_from_words(*w)[c % 4]) / np.sqrt(k)
    return out


def test_c2_bf16_sketch_sampled_outputs(api, ctx):
    """d = 200,000, n1 = n2 = 2,000, k = 400 in the benchmark's launch
    configuration: 16 sketch rows x 24 columns of A~ and B~ against the
    oracle's BF16 definition computed one by one."""
    c = smp_inputs.CONFIGS["c2_fp32"]
    log("c2 bf16 sketch sampled")
    Ad, Bd = smp_inputs.latent_pair(c["d"], c["n1"], c["n2"], c["R"], c["sigma"], c["alpha"], SEED, device=DEV)
    p = _bf16_params(api, c["d"], c["n1"], c["n2"], c["k"])
    At, Bt, na2, _ = _sketch_gpu(api, ctx, p, Ad, Bd, c["n1"], c["n2"], c["k"])
    rng = np.random.default_rng(1)
    rows_c = sorted(set(rng.choice(c["k"], 16, replace=False).tolist()) | {0, c["k"] - 1})
    cols = sorted(set(rng.choice(c["n1"], 24, replace=False).tolist()) | {0, c["n1"] - 1})
    P = _pi_rows_bf16(p.seed, c["k"], rows_c, c["d"])
    for X, S in ((Ad, At), (Bd, Bt)):
        Xs = rounding.round_bf16(X[:, cols].double().cpu().numpy())
        ref = P @ Xs
        got = S[cols][:, rows_c].astype(np.float64).T
        col_rel = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
        log(f"  max column rel {col_rel.max():.3e}")
        assert col_rel.max() < TOL_SKETCH
    ref_na2 = (Ad.double() ** 2).sum(0).cpu().numpy()
    assert np.allclose(na2, ref_na2, rtol=1e-6)


SOLVE_CASES = {
    "c1": dict(d=2000, n1=200, n2=200, R=5, k=50, r=5, T=10),
    "ragged": dict(d=1037, n1=77, n2=131, R=3, k=37, r=3, T=8),
    "k400_r10": dict(d=20000, n1=300, n2=260, R=10, k=400, r=10, T=10),
    "tiny_d1": dict(d=1, n1=3, n2=4, R=1, k=2, r=1, T=3),        # no whole 32-row block: tail launch only
    "single_row": dict(d=64, n1=1, n2=5, R=1, k=3, r=1, T=2),
}


@pytest.mark.parametrize("name", list(SOLVE_CASES))
def test_solve_bf16_matches_oracle(api, ctx, name):
    c = SOLVE_CASES[name]
    log(f"bf16 solve {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=c["R"])
    m = api.default_m(c["n1"], c["n2"], c["r"]) if min(c["n1"], c["n2"]) > 1 else 50.0
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], m=m, prec=api.SMP_PREC_BF16,
                        init_iters=40)
    U = torch.empty(c["n1"], c["r"], dtype=torch.float64, device=DEV)
    V = torch.empty(c["n2"], c["r"], dtype=torch.float64, device=DEV)
    s = torch.empty(c["r"], dtype=torch.float64, device=DEV)
    ctx.smp_solve(p, Ad, Bd, U, V, s)
    torch.cuda.synchronize()
    ref = oso.smp_pca(A.numpy(), B.numpy(), c["r"], c["k"], p.m, c["T"], SEED, sketch_fmt="bf16")
    AtB = oev.product(A.numpy(), B.numpy())
    e_gpu = oev.relative_error(AtB, U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy())
    e_ora = oev.relative_error(AtB, ref["Uc"], ref["sigma"], ref["Vc"])
    log(f"  e_gpu={e_gpu:.6e} e_oracle_bf16={e_ora:.6e}")
    # an exactly low-rank product (the rank-1 cases) leaves errors near FP32
    # rounding on both sides, which the relative term alone does not resolve
    assert abs(e_gpu - e_ora) <= 1e-3 * e_ora + 1e-6


def test_c2_bf16_solve_error_against_fp64_oracle(api, ctx):
    """The benchmark workload with the BF16 sketch: the spectral error stays
    within 1.02x of the FP64 oracle's (plain FP64 sketch)."""
    c = smp_inputs.CONFIGS["c2_fp32"]
    log("c2 bf16 end to end")
    Ad, Bd = smp_inputs.latent_pair(c["d"], c["n1"], c["n2"], c["R"], c["sigma"], c["alpha"], SEED, device=DEV)
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], prec=api.SMP_PREC_BF16)
    U = torch.empty(c["n1"], c["r"], dtype=torch.float64, device=DEV)
    V = torch.empty(c["n2"], c["r"], dtype=torch.float64, device=DEV)
    s = torch.empty(c["r"], dtype=torch.float64, device=DEV)
    ctx.smp_solve(p, Ad, Bd, U, V, s)
    torch.cuda.synchronize()
    A, B = Ad.cpu().numpy(), Bd.cpu().numpy()
    ref = oso.smp_pca(A, B, c["r"], c["k"], p.m, c["T"], SEED)
    AtB = oev.product(A, B)
    e_gpu = oev.relative_error(AtB, U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy())
    e_ora = oev.relative_error(AtB, ref["Uc"], ref["sigma"], ref["Vc"])
    log(f"  e_gpu_bf16={e_gpu:.6e} e_oracle_fp64={e_ora:.6e} ratio={e_gpu / e_ora:.4f}")
    assert e_gpu <= 1.02 * e_ora


# ---------------------------------------------------------------- FP8 E4M3 with E8M0 block scales
#
# Tolerance: the GPU rounds its FP32 Box-Muller draw to E4M3, the oracle its
# FP64 draw; they differ where the draw lies within a few FP32 ulps of an E4M3
# rounding midpoint (probability ~2^-17 per entry), each such entry moving its
# product by 2^-4 relative: sqrt(2^-17) * 2^-4 ~ 2e-4 of the column norm. The
# data side is identical on both sides (same FP32 values, exact power-of-two
# scaling, the same scale decisions). Gate 1e-3 per column.

TOL_FP8 = 1e-3

FP8_CASES = {
    "c1": dict(d=2000, n1=200, n2=200, k=50),
    "ragged": dict(d=1037, n1=77, n2=131, k=37),
    "k400_tiles": dict(d=20000, n1=300, n2=1100, k=400),
    "tiny": dict(d=3, n1=1, n2=5, k=1),
    "block_tail": dict(d=333, n1=512, n2=6, k=81),
}


@pytest.mark.parametrize("name", list(FP8_CASES))
def test_sketch_fp8_parity(api, ctx, name):
    c = FP8_CASES[name]
    log(f"fp8 sketch {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=min(5, c["n1"], c["n2"]))
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], r=1, prec=api.SMP_PREC_FP8)
    At, Bt, na2, nb2 = _sketch_gpu(api, ctx, p, Ad, Bd, c["n1"], c["n2"], c["k"])
    oAt, oBt, ona2, onb2 = osk.sketch_lowp(A.numpy(), B.numpy(), p.seed, c["k"], "fp8")
    ea, eb = _col_rel(At, oAt), _col_rel(Bt, oBt)
    log(f"  column rel err A {ea:.2e} B {eb:.2e}")
    assert ea < TOL_FP8 and eb < TOL_FP8
    assert np.allclose(na2, ona2, rtol=1e-6, atol=0)
    assert np.allclose(nb2, onb2, rtol=1e-6, atol=0)


@pytest.mark.parametrize("name", ["c1", "ragged", "k400_tiles"])
def test_sketch_fp8_regenerating_pass_parity(api, ctx, name, monkeypatch):
    """The FP8 pass that regenerates Pi inside each workgroup (selected with
    SMP_SKETCH_FP8_STORED=0; the default pass stores Pi once per push) meets the
    same bar against the oracle."""
    monkeypatch.setenv("SMP_SKETCH_FP8_STORED", "0")
    c = FP8_CASES[name]
    log(f"fp8 regenerating sketch {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=min(5, c["n1"], c["n2"]))
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], r=1, prec=api.SMP_PREC_FP8)
    At, Bt, na2, nb2 = _sketch_gpu(api, ctx, p, Ad, Bd, c["n1"], c["n2"], c["k"])
    oAt, oBt, ona2, onb2 = osk.sketch_lowp(A.numpy(), B.numpy(), p.seed, c["k"], "fp8")
    assert _col_rel(At, oAt) < TOL_FP8 and _col_rel(Bt, oBt) < TOL_FP8
    assert np.allclose(na2, ona2, rtol=1e-6, atol=0)
    assert np.allclose(nb2, onb2, rtol=1e-6, atol=0)


FP8_FRAG_CASES = dict(FP8_CASES, k1024_two_chunks=dict(d=1500, n1=70, n2=300, k=1024),
                      padded_ld=dict(d=700, n1=45, n2=33, k=500, ld_pad=3))


@pytest.mark.parametrize("name", list(FP8_FRAG_CASES))
def test_sketch_fp8_fragment_pass_parity(api, ctx, name, monkeypatch):
    """The FP8 pass that first quantises each window of rows into MFMA operand
    fragments (the default for k > 416; selected here with
    SMP_SKETCH_FP8_STORED=2 at every k) meets the oracle's FP8 bar: the same
    E8M0 block scales and E4M3 values, the norms of the unrounded data. Cases
    cover a single row, a partial last 128-row block (zero-padded), column
    counts that are not multiples of 16 or 256, two sketch-row chunks and a
    leading dimension larger than the column count."""
    monkeypatch.setenv("SMP_SKETCH_FP8_STORED", "2")
    c = FP8_FRAG_CASES[name]
    log(f"fp8 fragment sketch {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=min(5, c["n1"], c["n2"]))
    pad = c.get("ld_pad", 0)
    if pad:   # the same values at a leading dimension of n + pad
        Ad = torch.zeros(c["d"], c["n1"] + pad, device=DEV)[:, :c["n1"]].copy_(Ad)
        Bd = torch.zeros(c["d"], c["n2"] + pad, device=DEV)[:, :c["n2"]].copy_(Bd)
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], r=1, prec=api.SMP_PREC_FP8)
    At, Bt, na2, nb2 = _sketch_gpu(api, ctx, p, Ad, Bd, c["n1"], c["n2"], c["k"])
    oAt, oBt, ona2, onb2 = osk.sketch_lowp(A.numpy(), B.numpy(), p.seed, c["k"], "fp8")
    ea, eb = _col_rel(At, oAt), _col_rel(Bt, oBt)
    log(f"  column rel err A {ea:.2e} B {eb:.2e}")
    assert ea < TOL_FP8 and eb < TOL_FP8
    assert np.allclose(na2, ona2, rtol=1e-6, atol=0)
    assert np.allclose(nb2, onb2, rtol=1e-6, atol=0)


def test_sketch_fp8_fragment_pass_windows_and_pushes(api, ctx, monkeypatch):
    """The fragment pass over many windows (1 MiB: a few 128-row blocks each)
    and as streaming pushes out of order, starting and ending inside 128-row
    blocks (whole 32-row blocks only): both meet the oracle's bar and agree
    with the one-window pass up to the FP32 rounding of the partial sums."""
    monkeypatch.setenv("SMP_SKETCH_FP8_STORED", "2")
    d, n1, n2, k = 5000, 130, 70, 640
    A, B, Ad, Bd = latent(d, n1, n2)
    oAt, oBt, ona2, onb2 = osk.sketch_lowp(A.numpy(), B.numpy(), SEED, k, "fp8")
    p = api.make_params(d, n1, n2, k, r=1, prec=api.SMP_PREC_FP8, seed=SEED)
    outs = []
    for mb in ("4096", "1"):
        monkeypatch.setenv("SMP_PI_WINDOW_MB", mb)
        outs.append(_sketch_gpu(api, ctx, p, Ad, Bd, n1, n2, k))
    st = ctx.smp_sketch_begin(p)
    for l0, l1 in [(2080, 5000), (0, 32), (32, 2080)]:
        ctx.smp_sketch_push(st, Ad[l0:l1], Bd[l0:l1], l0)
    At = torch.empty(n1, k, device=DEV)
    Bt = torch.empty(n2, k, device=DEV)
    na2 = torch.empty(n1, device=DEV)
    nb2 = torch.empty(n2, device=DEV)
    ctx.smp_sketch_end(st, At, Bt, na2, nb2)
    torch.cuda.synchronize()
    ctx.smp_sketch_free(st)
    outs.append((At.cpu().numpy(), Bt.cpu().numpy(), na2.cpu().numpy(), nb2.cpu().numpy()))
    for Ao, Bo, na, nb in outs:
        assert _col_rel(Ao, oAt) < TOL_FP8 and _col_rel(Bo, oBt) < TOL_FP8
        assert np.allclose(na, ona2, rtol=1e-6, atol=0) and np.allclose(nb, onb2, rtol=1e-6, atol=0)
    for Ao, Bo, _, _ in outs[1:]:
        assert _col_rel(Ao, outs[0][0].T.astype(np.float64)) < 1e-6
        assert _col_rel(Bo, outs[0][1].T.astype(np.float64)) < 1e-6


def test_sketch_fp8_fragment_pass_b_is_a(api, ctx, monkeypatch):
    """The fragment pass for B = A (the PCA case): only A's n-tiles are
    quantised (no B matrix), one-shot and as out-of-order streaming pushes,
    with a column count that is not a multiple of 16 and a partial last
    128-row block; the sketch meets the oracle's FP8 bar and B~ = A~."""
    monkeypatch.setenv("SMP_SKETCH_FP8_STORED", "2")
    d, n, k = 1500, 150, 640
    A, _, Ad, _ = latent(d, n, n, same=True)
    p = api.make_params(d, n, n, k, r=1, prec=api.SMP_PREC_FP8, b_is_a=True)
    oAt, _, ona2, _ = osk.sketch_lowp(A.numpy(), None, p.seed, k, "fp8")
    log(f"fp8 fragment sketch B = A d={d} n={n} k={k}")
    outs = []
    for mode in ("one-shot", "pushes"):
        At = torch.empty(n, k, device=DEV)
        Bt = torch.empty(n, k, device=DEV)
        na2 = torch.empty(n, device=DEV)
        nb2 = torch.empty(n, device=DEV)
        if mode == "one-shot":
            ctx.smp_sketch(p, Ad, None, At, Bt, na2, nb2)
        else:
            st = ctx.smp_sketch_begin(p)
            for l0, l1 in [(640, 1500), (0, 64), (64, 640)]:
                ctx.smp_sketch_push(st, Ad[l0:l1], None, l0)
            ctx.smp_sketch_end(st, At, Bt, na2, nb2)
        torch.cuda.synchronize()
        if mode == "pushes":
            ctx.smp_sketch_free(st)
        assert torch.equal(At, Bt) and torch.equal(na2, nb2)
        e = _col_rel(At.cpu().numpy(), oAt)
        log(f"  {mode}: column rel err {e:.2e}")
        assert e < TOL_FP8
        assert np.allclose(na2.cpu().numpy(), ona2, rtol=1e-6, atol=0)
        outs.append(At.cpu().numpy())
    assert _col_rel(outs[1], outs[0].T.astype(np.float64)) < 1e-6


def test_sketch_fp8_streaming_push_on_block_boundaries(api, ctx):
    d, n1, n2, k = 3000, 130, 70, 64
    A, B, Ad, Bd = latent(d, n1, n2)
    p = api.make_params(d, n1, n2, k, r=1, prec=api.SMP_PREC_FP8)
    st = ctx.smp_sketch_begin(p)
    with pytest.raises(api.SmpError):
        ctx.smp_sketch_push(st, Ad[0:40], Bd[0:40], 0)          # 40 rows: not whole 32-row blocks
    for l0, l1 in [(2016, 3000), (0, 32), (32, 2016)]:
        ctx.smp_sketch_push(st, Ad[l0:l1], Bd[l0:l1], l0)
    At = torch.empty(n1, k, device=DEV)
    Bt = torch.empty(n2, k, device=DEV)
    na2 = torch.empty(n1, device=DEV)
    nb2 = torch.empty(n2, device=DEV)
    ctx.smp_sketch_end(st, At, Bt, na2, nb2)
    torch.cuda.synchronize()
    ctx.smp_sketch_free(st)
    oAt, oBt, _, _ = osk.sketch_lowp(A.numpy(), B.numpy(), p.seed, k, "fp8")
    assert _col_rel(At.cpu().numpy(), oAt) < TOL_FP8
    assert _col_rel(Bt.cpu().numpy(), oBt) < TOL_FP8


def test_solve_fp8_matches_oracle_and_reports_error(api, ctx):
    c = dict(d=20000, n1=300, n2=260, R=10, k=400, r=10, T=10)
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=c["R"])
    m = api.default_m(c["n1"], c["n2"], c["r"])
    res = {}
    for name, prec in (("fp8", api.SMP_PREC_FP8), ("fp32", api.SMP_PREC_FP32)):
        p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], m=m, prec=prec, init_iters=40)
        U = torch.empty(c["n1"], c["r"], dtype=torch.float64, device=DEV)
        V = torch.empty(c["n2"], c["r"], dtype=torch.float64, device=DEV)
        s = torch.empty(c["r"], dtype=torch.float64, device=DEV)
        ctx.smp_solve(p, Ad, Bd, U, V, s)
        torch.cuda.synchronize()
        res[name] = (U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy(), p)
    AtB = oev.product(A.numpy(), B.numpy())
    ref8 = oso.smp_pca(A.numpy(), B.numpy(), c["r"], c["k"], res["fp8"][3].m, c["T"], SEED, sketch_fmt="fp8")
    e8 = oev.relative_error(AtB, *res["fp8"][:3])
    e32 = oev.relative_error(AtB, *res["fp32"][:3])
    e8_ora = oev.relative_error(AtB, ref8["Uc"], ref8["sigma"], ref8["Vc"])
    log(f"  e_fp8={e8:.6e} e_oracle_fp8={e8_ora:.6e} e_fp32={e32:.6e}")
    assert abs(e8 - e8_ora) <= 5e-3 * e8_ora


FP8_SOLVE_CASES = {
    "ragged": dict(d=1037, n1=77, n2=131, R=3, k=37, r=3, T=8),
    "tiny_d1": dict(d=1, n1=3, n2=4, R=1, k=2, r=1, T=3),        # no whole 32-row block: tail launch only
    "single_row": dict(d=64, n1=1, n2=5, R=1, k=3, r=1, T=2),
}


@pytest.mark.parametrize("name", list(FP8_SOLVE_CASES))
def test_solve_fp8_small_and_degenerate(api, ctx, name):
    """FP8 solve against the oracle's FP8 pipeline on a ragged shape and the
    degenerate ones (a single data row, a single column of A)."""
    c = FP8_SOLVE_CASES[name]
    log(f"fp8 solve {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=c["R"])
    m = api.default_m(c["n1"], c["n2"], c["r"]) if min(c["n1"], c["n2"]) > 1 else 50.0
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], m=m, prec=api.SMP_PREC_FP8,
                        init_iters=40)
    U = torch.empty(c["n1"], c["r"], dtype=torch.float64, device=DEV)
    V = torch.empty(c["n2"], c["r"], dtype=torch.float64, device=DEV)
    s = torch.empty(c["r"], dtype=torch.float64, device=DEV)
    ctx.smp_solve(p, Ad, Bd, U, V, s)
    torch.cuda.synchronize()
    ref = oso.smp_pca(A.numpy(), B.numpy(), c["r"], c["k"], p.m, c["T"], SEED, sketch_fmt="fp8")
    AtB = oev.product(A.numpy(), B.numpy())
    e_gpu = oev.relative_error(AtB, U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy())
    e_ora = oev.relative_error(AtB, ref["Uc"], ref["sigma"], ref["Vc"])
    log(f"  e_gpu={e_gpu:.6e} e_oracle_fp8={e_ora:.6e}")
    assert abs(e_gpu - e_ora) <= 5e-3 * e_ora + 1e-6


def _pi_rows_e4m3(seed, k, rows_c, d):
    """E(Z(c, l)) / sqrt(k) for selected sketch rows c and all l < d."""
    out = np.empty((len(rows_c), d))
    ls = np.arange(d, dtype=np.int64)
    for t, c in enumerate(rows_c):
        w = philox.stream_words(seed, philox.TAG_PI, ls, np.full(d, c // 4, dtype=np.int64))
        out[t] = rounding.round_e4m3(gaussian.normals_from_words(*w)[c % 4]) / np.sqrt(k)
    return out


def test_c2_fp8_sketch_sampled_outputs(api, ctx):
    """d = 200,000, n1 = n2 = 2,000, k = 400 with the FP8 pass in the
    benchmark's launch configuration: 16 sketch rows x 24 columns of A~ and B~
    against the oracle's FP8 definition (E4M3 Pi, E4M3 data with E8M0 scales
    per column and 32-row block) computed one by one."""
    c = smp_inputs.CONFIGS["c2_fp32"]
    log("c2 fp8 sketch sampled")
    Ad, Bd = smp_inputs.latent_pair(c["d"], c["n1"], c["n2"], c["R"], c["sigma"], c["alpha"], SEED, device=DEV)
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], r=1, prec=api.SMP_PREC_FP8)
    At, Bt, na2, _ = _sketch_gpu(api, ctx, p, Ad, Bd, c["n1"], c["n2"], c["k"])
    rng = np.random.default_rng(2)
    rows_c = sorted(set(rng.choice(c["k"], 16, replace=False).tolist()) | {0, c["k"] - 1})
    cols = sorted(set(rng.choice(c["n1"], 24, replace=False).tolist()) | {0, c["n1"] - 1})
    P = _pi_rows_e4m3(p.seed, c["k"], rows_c, c["d"])
    for X, S in ((Ad, At), (Bd, Bt)):
        Xs = rounding.quantize_e4m3_blocks(X[:, cols].double().cpu().numpy())
        ref = P @ Xs
        got = S[cols][:, rows_c].astype(np.float64).T
        col_rel = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
        log(f"  max column rel {col_rel.max():.3e}")
        assert col_rel.max() < TOL_FP8
    ref_na2 = (Ad.double() ** 2).sum(0).cpu().numpy()
    assert np.allclose(na2, ref_na2, rtol=1e-6)

"""smp_tune_sketch on the GPU: it times the launch shapes of the sketch pass,
stores the fastest in the process-wide table, and every later sketch of that
shape uses it. The tuned pass is still the oracle's sketch (same bars as the
untuned passes) and differs from the untuned one only by the FP32 rounding of
the split-K sums."""

import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_common import DEV, latent, log
from oracle import sketch as osk

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def api():
    from paper_1610_06656_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def _sketch(ctx, p, Ad, Bd, n1, n2, k):
    out = [torch.empty(n1, k, device=DEV), torch.empty(n2, k, device=DEV), torch.empty(n1, device=DEV),
           torch.empty(n2, device=DEV)]
    ctx.smp_sketch(p, Ad, Bd, *out)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in out]


def _col_rel(got_t, ref):
    g = got_t.T.astype(np.float64)
    return float(np.max(np.linalg.norm(g - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)))


@pytest.mark.parametrize("prec_name", ["bf16", "fp32", "fp8"])
def test_tuned_sketch_is_the_oracles(api, ctx, prec_name, tmp_path):
    api.smp_tune_clear()
    prec = {"bf16": api.SMP_PREC_BF16, "fp32": api.SMP_PREC_FP32, "fp8": api.SMP_PREC_FP8}[prec_name]
    d, n1, n2, k = 9000, 300, 170, 300
    A, B, Ad, Bd = latent(d, n1, n2)
    p = api.make_params(d, n1, n2, k, r=1, prec=prec)
    before = _sketch(ctx, p, Ad, Bd, n1, n2, k)
    cap, splits, ms = ctx.smp_tune_sketch(p, Ad, Bd)
    log(f"{prec_name}: tuned cap {cap} splits {splits} {ms:.3f} ms")
    assert splits >= 1 and ms > 0 and (cap in (13, 16) if prec_name == "bf16" else cap == 0)
    assert api.smp_tune_lookup(p) == (cap, splits)
    after = _sketch(ctx, p, Ad, Bd, n1, n2, k)
    fmt = {"bf16": "bf16", "fp8": "fp8", "fp32": None}[prec_name]
    if fmt:
        oA, oB, ona, onb = osk.sketch_lowp(A.numpy(), B.numpy(), p.seed, k, fmt)
    else:
        oA, oB, ona, onb = osk.sketch(A.numpy(), B.numpy(), p.seed, k)
    tol = {"bf16": 2e-4, "fp32": 1e-5, "fp8": 1e-3}[prec_name]
    assert _col_rel(after[0], oA) < tol and _col_rel(after[1], oB) < tol
    assert np.allclose(after[2], ona, rtol=1e-6) and np.allclose(after[3], onb, rtol=1e-6)
    for a, b in zip(before[:2], after[:2]):        # the same sums in another split: FP32 rounding only
        assert _col_rel(a, b.T.astype(np.float64)) < 1e-5
    # the table round-trips through its file and keeps steering the pass
    api.smp_tune_save(tmp_path / "tune.json")
    api.smp_tune_clear()
    assert api.smp_tune_lookup(p) == (0, 0)
    api.smp_tune_load(tmp_path / "tune.json")
    again = _sketch(ctx, p, Ad, Bd, n1, n2, k)
    for a, b in zip(after, again):
        assert np.array_equal(a, b)
    api.smp_tune_clear()


def test_tune_b_is_a_and_streaming_state(api, ctx):
    api.smp_tune_clear()
    d, n, k = 12000, 256, 256
    A, _, Ad, _ = latent(d, n, n, same=True)
    p = api.make_params(d, n, n, k, r=1, prec=api.SMP_PREC_BF16, b_is_a=True)
    cap, splits, ms = ctx.smp_tune_sketch(p, Ad, None)
    assert api.smp_tune_lookup(p) == (cap, splits)
    assert api.smp_tune_lookup(api.make_params(d, n, n, k, r=1, prec=api.SMP_PREC_BF16)) == (0, 0)
    one = _sketch(ctx, p, Ad, None, n, n, k)
    st = ctx.smp_sketch_begin(p)            # a streaming state of the tuned shape uses the tuned launch too
    ctx.smp_sketch_push(st, Ad, None, 0)
    out = [torch.empty(n, k, device=DEV), torch.empty(n, k, device=DEV), torch.empty(n, device=DEV),
           torch.empty(n, device=DEV)]
    ctx.smp_sketch_end(st, *out)
    torch.cuda.synchronize()
    ctx.smp_sketch_free(st)
    assert _col_rel(out[0].cpu().numpy(), one[0].T.astype(np.float64)) < 1e-5
    oA, _, _, _ = osk.sketch_lowp(A.numpy(), None, p.seed, k, "bf16")
    assert _col_rel(one[0], oA) < 2e-4
    with pytest.raises(api.SmpError):
        ctx.smp_tune_sketch(api.make_params(d, n, n, k, r=1, sketch="srht"), Ad, Ad)
    api.smp_tune_clear()

"""GPU parity of the SRHT sketch (SMP_SKETCH_SRHT; the paper's Spark sketch,
Section 4) against the oracle's definition (oracle.srht: Pi formed block by
block and multiplied in FP64). The GPU computes the same product by fast
Walsh-Hadamard transforms of 512-row chunks in FP32.

Tolerances: per column ||dA~_i|| / ||A~_i|| <= 1e-5 (FP32 additions: nine
butterfly levels per chunk, then one sum over the chunks per split and an FP64
reduction of the splits); norms 1e-6; the solve's spectral error within 1e-4
(relative) of the oracle's with the same sketch.
"""

import numpy as np
import pytest
import torch

import smp_inputs
from conftest import gpu_available
from gpu_common import DEV, SEED, latent, log
from oracle import evaluate as oev
from oracle import solve as oso
from oracle import srht as osr

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def api():
    from paper_1610_06656_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def _col_rel(got_t, ref):
    g = got_t.T.astype(np.float64)
    return float(np.max(np.linalg.norm(g - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)))


CASES = {
    "c1": dict(d=2000, n1=200, n2=200, k=50),
    "ragged": dict(d=1037, n1=77, n2=131, k=37),
    "k400": dict(d=20000, n1=300, n2=1100, k=400),
    "k1500_two_blocks": dict(d=3000, n1=129, n2=64, k=1500),
    "tiny": dict(d=3, n1=1, n2=5, k=1),
    "pow2": dict(d=4096, n1=40, n2=33, k=64),
    "one_row_past_chunk": dict(d=513, n1=70, n2=45, k=20),
}


def _sketch(api, ctx, p, Ad, Bd, n1, n2, k):
    At = torch.empty(n1, k, device=DEV)
    Bt = torch.empty(n2, k, device=DEV)
    na2 = torch.empty(n1, device=DEV)
    nb2 = torch.empty(n2, device=DEV)
    ctx.smp_sketch(p, Ad, Bd, At, Bt, na2, nb2)
    torch.cuda.synchronize()
    return At.cpu().numpy(), Bt.cpu().numpy(), na2.cpu().numpy(), nb2.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_srht_sketch_parity(api, ctx, name):
    c = CASES[name]
    log(f"srht sketch {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=min(5, c["n1"], c["n2"]))
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], r=1, sketch="srht")
    At, Bt, na2, nb2 = _sketch(api, ctx, p, Ad, Bd, c["n1"], c["n2"], c["k"])
    oAt, oBt, ona2, onb2 = osr.sketch(A.numpy(), B.numpy(), SEED, c["k"])
    ea, eb = _col_rel(At, oAt), _col_rel(Bt, oBt)
    log(f"  column rel err A {ea:.2e} B {eb:.2e}")
    assert ea < 1e-5 and eb < 1e-5
    assert np.allclose(na2, ona2, rtol=1e-6, atol=0) and np.allclose(nb2, onb2, rtol=1e-6, atol=0)


def test_srht_streaming_pushes_split_chunks(api, ctx):
    """Pushes that start and end inside 512-row chunks, out of order; and the
    PCA case B = A."""
    d, n1, n2, k = 5000, 90, 70, 100
    A, B, Ad, Bd = latent(d, n1, n2)
    p = api.make_params(d, n1, n2, k, r=1, sketch="srht")
    st = ctx.smp_sketch_begin(p)
    for l0, l1 in [(3001, 5000), (0, 700), (700, 3001)]:
        ctx.smp_sketch_push(st, Ad[l0:l1], Bd[l0:l1], l0)
    At = torch.empty(n1, k, device=DEV)
    Bt = torch.empty(n2, k, device=DEV)
    na2 = torch.empty(n1, device=DEV)
    nb2 = torch.empty(n2, device=DEV)
    ctx.smp_sketch_end(st, At, Bt, na2, nb2)
    torch.cuda.synchronize()
    ctx.smp_sketch_free(st)
    oAt, oBt, ona2, _ = osr.sketch(A.numpy(), B.numpy(), SEED, k)
    assert _col_rel(At.cpu().numpy(), oAt) < 1e-5 and _col_rel(Bt.cpu().numpy(), oBt) < 1e-5
    assert np.allclose(na2.cpu().numpy(), ona2, rtol=1e-6)
    # B = A
    p2 = api.make_params(d, n1, n1, k, r=1, sketch="srht", b_is_a=True)
    At2 = torch.empty(n1, k, device=DEV)
    Bt2 = torch.empty(n1, k, device=DEV)
    na = torch.empty(n1, device=DEV)
    nb = torch.empty(n1, device=DEV)
    ctx.smp_sketch(p2, Ad, None, At2, Bt2, na, nb)
    torch.cuda.synchronize()
    oAt2, _, _, _ = osr.sketch(A.numpy(), None, SEED, k)
    assert _col_rel(At2.cpu().numpy(), oAt2) < 1e-5 and torch.equal(At2, Bt2)


def test_srht_rejects_low_precision(api):
    p = api.make_params(1000, 10, 10, 8, 2, sketch="srht", prec=api.SMP_PREC_BF16)
    with pytest.raises(api.SmpError):
        api.smp_check_params(p)


def test_srht_solve_matches_oracle(api, ctx):
    c = smp_inputs.CONFIGS["c1_small"]
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=c["R"], sigma=c["sigma"], alpha=c["alpha"])
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], init_iters=40, sketch="srht")
    U = torch.empty(c["n1"], c["r"], dtype=torch.float64, device=DEV)
    V = torch.empty(c["n2"], c["r"], dtype=torch.float64, device=DEV)
    s = torch.empty(c["r"], dtype=torch.float64, device=DEV)
    ctx.smp_solve(p, Ad, Bd, U, V, s)
    torch.cuda.synchronize()
    M = oev.product(A.numpy(), B.numpy())
    e = oev.relative_error(M, U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy())
    ref = oso.smp_pca(A.numpy(), B.numpy(), c["r"], c["k"], p.m, c["T"], SEED, sketch_kind="srht")
    eo = oev.relative_error(M, ref["Uc"], ref["sigma"], ref["Vc"])
    log(f"  srht solve error gpu {e:.6e} oracle {eo:.6e}")
    assert abs(e - eo) <= 1e-4 * eo

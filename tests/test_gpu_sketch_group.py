"""GPU parity of smp_sketch_group (the sketches of many independent BF16 jobs
in grouped launches; Alg. 1 step 2 for each job) against the oracle's BF16
definition of each job's sketch (``sketch_lowp``), and against each job's
own regenerating pass.

Tolerances: per column ||dA~_i|| / ||A~_i|| <= 2e-4 against the oracle (the
BF16 bar of the single-job sketch tests: the FP32 and FP64 draws of Pi round
to different bfloat16 values on ~2^-14 of the entries), squared norms 1e-6
relative (unrounded FP32 data, compensated sums); against the job's own pass
1e-5 per column: the same products, with the rows cut into other split-K
partials, so the FP32 accumulators add them in another order (one rounding of
~6e-8 per 32-row step of a running sum: ~4e-8 sqrt(d / 32) of the column
norm per order, 1.4e-6 at d = 20,000 for the difference of two).
"""

import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_common import DEV, SEED, latent, log
from oracle import sketch as osk

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL_SKETCH = 2e-4

# (d, n1, n2, k, B = A, leading-dimension padding): ragged and aligned column
# counts, k on both tile shapes of the pass (k <= 448: 4 columns per lane and
# up to 4 m-tiles; larger k: 2 columns and up to 12 m-tiles), d with and
# without a partial last 128-row block, with fewer rows than one block, with
# enough blocks for several row splits, B = A, and an odd leading dimension
# (the scalar-load kernel)
JOBS = [
    (2000, 200, 200, 50, False, 0),
    (1037, 77, 131, 37, False, 0),
    (20000, 300, 260, 400, False, 0),
    (3, 1, 5, 1, False, 0),
    (100, 33, 64, 20, False, 0),
    (9000, 128, 256, 20, False, 0),
    (1500, 96, 96, 40, True, 0),
    (700, 45, 33, 21, False, 3),
    (4096, 129, 64, 1024, False, 0),
    (2048, 64, 64, 100, True, 0),
    (1037, 77, 131, 37, False, 0),
    (20000, 512, 512, 400, False, 0),
]


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


def _inputs(api, idx, d, n1, n2, k, same, pad):
    A, B, _, _ = latent(d, n1, n2, R=min(5, n1, n2), seed=SEED + idx, same=same)
    Ad = torch.zeros(d, n1 + pad, device=DEV)[:, :n1].copy_(A.to(DEV)) if pad else A.to(DEV)
    Bd = None if same else B.to(DEV)
    p = api.make_params(d, n1, n2, k, r=1, prec=api.SMP_PREC_BF16, seed=SEED + 100 + idx, b_is_a=same)
    return A, (A if same else B), Ad, Bd, p


def test_sketch_group_matches_oracle_and_each_jobs_own_pass(api, ctx, monkeypatch):
    jobs = [_inputs(api, i, *j) for i, j in enumerate(JOBS)]
    outs = []
    for i, ((d, n1, n2, k, same, pad), (A, B, Ad, Bd, p)) in enumerate(zip(JOBS, jobs)):
        outs.append((torch.full((n1, k), float("nan"), device=DEV), torch.full((n2, k), float("nan"), device=DEV),
                     torch.full((n1,), float("nan"), device=DEV), torch.full((n2,), float("nan"), device=DEV)))
    log(f"sketch group of {len(jobs)} jobs")
    ctx.smp_sketch_group([j[4] for j in jobs], [j[2] for j in jobs], [j[3] for j in jobs],
                         [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs], [o[3] for o in outs])
    torch.cuda.synchronize()
    monkeypatch.setenv("SMP_SKETCH_BF16_STORED", "0")   # each job's own regenerating pass
    own_ctx = api.Context(0)
    for i, ((d, n1, n2, k, same, pad), (A, B, Ad, Bd, p), (At, Bt, na2, nb2)) in enumerate(zip(JOBS, jobs, outs)):
        oAt, oBt, ona2, onb2 = osk.sketch_lowp(A.numpy(), None if same else B.numpy(), p.seed, k, "bf16")
        if same:
            oBt, onb2 = oAt, ona2
        ea, eb = _col_rel(At.cpu().numpy(), oAt), _col_rel(Bt.cpu().numpy(), oBt)
        log(f"  job {i} d={d} n1={n1} n2={n2} k={k} same={same} pad={pad}: column rel err A {ea:.2e} B {eb:.2e}")
        assert ea < TOL_SKETCH and eb < TOL_SKETCH
        assert np.allclose(na2.cpu().numpy(), ona2, rtol=1e-6, atol=0)
        assert np.allclose(nb2.cpu().numpy(), onb2, rtol=1e-6, atol=0)
        if same:
            assert torch.equal(At, Bt) and torch.equal(na2, nb2)
        sAt = torch.empty(n1, k, device=DEV)
        sBt = torch.empty(n2, k, device=DEV)
        sna = torch.empty(n1, device=DEV)
        snb = torch.empty(n2, device=DEV)
        own_ctx.smp_sketch(p, Ad, Bd, sAt, sBt, sna, snb)
        torch.cuda.synchronize()
        assert _col_rel(At.cpu().numpy(), sAt.cpu().numpy().T.astype(np.float64)) < 1e-5
        assert _col_rel(Bt.cpu().numpy(), sBt.cpu().numpy().T.astype(np.float64)) < 1e-5
        assert np.allclose(na2.cpu().numpy(), sna.cpu().numpy(), rtol=1e-6, atol=0)


def test_sketch_group_repeated_calls_and_a_smaller_group(api, ctx):
    """The context's workspace is reused: a second call with fewer, smaller
    jobs gives the same values as those jobs had in the first call."""
    sel = [1, 4, 6]
    jobs = [_inputs(api, i, *JOBS[i]) for i in range(len(JOBS))]
    def run(idx):
        outs = []
        for i in idx:
            d, n1, n2, k, same, pad = JOBS[i]
            outs.append((torch.empty(n1, k, device=DEV), torch.empty(n2, k, device=DEV),
                         torch.empty(n1, device=DEV), torch.empty(n2, device=DEV)))
        ctx.smp_sketch_group([jobs[i][4] for i in idx], [jobs[i][2] for i in idx], [jobs[i][3] for i in idx],
                             [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs], [o[3] for o in outs])
        torch.cuda.synchronize()
        return outs
    first = run(list(range(len(JOBS))))
    second = run(sel)
    for o2, i in zip(second, sel):
        for a, b in zip(first[i], o2):
            assert torch.equal(a, b)


def test_sketch_group_rejects_other_precisions_and_accepts_no_jobs(api, ctx):
    d, n1, n2, k = 500, 20, 30, 16
    A, B, Ad, Bd = latent(d, n1, n2)
    At, Bt = torch.empty(n1, k, device=DEV), torch.empty(n2, k, device=DEV)
    na, nb = torch.empty(n1, device=DEV), torch.empty(n2, device=DEV)
    ctx.smp_sketch_group([], [], [], [], [], [], [])
    for prec in (api.SMP_PREC_FP32, api.SMP_PREC_FP8):
        p = api.make_params(d, n1, n2, k, r=1, prec=prec)
        with pytest.raises(api.SmpError):
            ctx.smp_sketch_group([p], [Ad], [Bd], [At], [Bt], [na], [nb])
    p = api.make_params(d, n1, n2, k, r=1, prec=api.SMP_PREC_BF16)
    with pytest.raises(api.SmpError):   # B missing without SMP_B_IS_A
        ctx.smp_sketch_group([p], [Ad], [None], [At], [Bt], [na], [nb])

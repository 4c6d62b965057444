"""WAltMin for a group of jobs (smp_waltmin_group): each job's result is
smp_waltmin's for that job bit for bit, with the grouped launches run eagerly
or as one HIP graph per group of equal launch sequences, whatever the other
jobs of the group are (shapes, r, T, subset mode), and on repeated calls with
eager work between them."""

import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_common import DEV, latent, log

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def api():
    from paper_1610_06656_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


JOBS = [  # d, n1, n2, k, r, T, split, seed offset
    (3000, 120, 90, 40, 3, 6, False, 0),
    (2500, 200, 150, 60, 5, 10, False, 1),
    (4000, 300, 260, 80, 10, 10, False, 2),
    (2000, 96, 130, 50, 5, 10, False, 3),     # same r and T as job 1: the same group
    (3500, 180, 200, 80, 20, 4, False, 4),    # r = 20: two-tile least squares
    (3000, 150, 120, 60, 5, 6, True, 5),      # SPLIT subsets
    (1500, 64, 40, 30, 10, 3, False, 6),
]


def _prepare(api, ctx, job):
    d, n1, n2, k, r, T, split, off = job
    A, B, Ad, Bd = latent(d, n1, n2, R=min(5, r), seed=7000 + off)
    p = api.make_params(d, n1, n2, k, r, T=T, init_iters=3, seed=99 + off,
                        omega_mode=api.SMP_OMEGA_SPLIT if split else api.SMP_OMEGA_REUSE)
    At = torch.empty(n1, k, device=DEV)
    Bt = torch.empty(n2, k, device=DEV)
    na2 = torch.empty(n1, device=DEV)
    nb2 = torch.empty(n2, device=DEV)
    ctx.smp_sketch(p, Ad, Bd, At, Bt, na2, nb2)
    om = api.Omega(n1, n2, int(p.m + 6 * p.m ** 0.5 + 64), DEV, split=split)
    ctx.smp_sample(p, na2, nb2, om)
    ctx.smp_estimate(p, At, Bt, na2, nb2, om)
    torch.cuda.synchronize()
    return p, om, na2


def _outs(n1, n2, r):
    return (torch.full((n1, r), np.nan, dtype=torch.float64, device=DEV),
            torch.full((n2, r), np.nan, dtype=torch.float64, device=DEV),
            torch.full((r,), np.nan, dtype=torch.float64, device=DEV))


@pytest.fixture(scope="module")
def prepared(api, ctx):
    jobs = [_prepare(api, ctx, j) for j in JOBS]
    ref = []
    for p, om, na2 in jobs:
        U, V, s = _outs(p.n1, p.n2, p.r)
        ctx.smp_waltmin(p, om, na2, U, V, s)
        torch.cuda.synchronize()
        ref.append((U.cpu().numpy(), V.cpu().numpy(), s.cpu().numpy()))
    return jobs, ref


@pytest.mark.parametrize("graph", [False, True])
def test_group_equals_each_job_alone(api, ctx, prepared, graph):
    jobs, ref = prepared
    outs = [_outs(p.n1, p.n2, p.r) for p, _, _ in jobs]
    ctx.smp_waltmin_group([j[0] for j in jobs], [j[1] for j in jobs], [j[2] for j in jobs],
                          [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs], graph=graph)
    for i, (o, rf) in enumerate(zip(outs, ref)):
        for a, b in zip(o, rf):
            assert np.array_equal(a.cpu().numpy(), b), f"job {i}"
    log(f"group of {len(jobs)} jobs (graph={graph}): identical to the jobs run alone")


def test_group_repeated_with_eager_work_between(api, ctx, prepared):
    """Three grouped calls in a row on different subsets, with other kernels and
    synchronisations between them; every result is the job's alone."""
    jobs, ref = prepared
    for subset, graph in (([6, 2, 0], True), ([1, 3, 5, 4], True), (list(range(len(jobs)))[::-1], False)):
        x = torch.randn(1 << 20, device=DEV)
        (x * 2).sum().item()                        # eager work and a synchronisation
        sel = [jobs[i] for i in subset]
        outs = [_outs(p.n1, p.n2, p.r) for p, _, _ in sel]
        ctx.smp_waltmin_group([j[0] for j in sel], [j[1] for j in sel], [j[2] for j in sel],
                              [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs], graph=graph)
        for i, o in zip(subset, outs):
            for a, b in zip(o, ref[i]):
                assert np.array_equal(a.cpu().numpy(), b), f"job {i} in {subset}"


def test_group_without_sigma_and_errors(api, ctx, prepared):
    jobs, ref = prepared
    p, om, na2 = jobs[2]
    U, V, _ = _outs(p.n1, p.n2, p.r)
    ctx.smp_waltmin_group([p], [om], [na2], [U], [V], None, graph=True)
    U1, V1, _ = _outs(p.n1, p.n2, p.r)
    ctx.smp_waltmin(p, om, na2, U1, V1, None)
    torch.cuda.synchronize()
    assert torch.equal(U, U1) and torch.equal(V, V1)
    bad = api.make_params(p.d, p.n1 + 1, p.n2, p.k, p.r)
    with pytest.raises(api.SmpError):
        ctx.smp_waltmin_group([bad], [om], [na2], [U], [V], None)
    ctx.smp_waltmin_group([], [], [], [], [], None)   # an empty group is a no-op

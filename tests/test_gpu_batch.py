"""GPU tests of batching and serving (smp_server_*, smp_solve_batch): every
job's result is bit-identical to the same job solved alone (the kernels are
deterministic and a job's arithmetic does not depend on what runs beside it),
jobs overlap on the device, the HBM budget bounds admission, and small jobs in
a batch match the oracle as smp_solve does."""

import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_common import DEV, SEED, latent, log
from oracle import evaluate as oev
from oracle import solve as oso

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def api():
    from paper_1610_06656_amd import api as a
    return a


# (d, n1, n2, k, r, T, prec, same)
JOBS = [
    (3000, 120, 90, 40, 4, 6, 0, False),
    (5000, 200, 200, 64, 5, 8, 1, False),
    (2500, 77, 131, 37, 3, 5, 0, False),
    (8000, 300, 260, 120, 10, 10, 1, False),
    (4000, 150, 150, 50, 5, 5, 0, True),
    (12000, 512, 384, 96, 8, 6, 1, False),
    (1037, 64, 64, 33, 2, 4, 1, True),
    (6000, 256, 128, 80, 6, 10, 0, False),
    (20000, 640, 520, 200, 10, 10, 1, False),
    (3500, 96, 200, 48, 4, 7, 0, False),
]


def _make(api, i, job):
    d, n1, n2, k, r, T, prec, same = job
    A, B, Ad, Bd = latent(d, n1, n2, R=max(1, r // 2), seed=SEED + 17 * i, same=same)
    p = api.make_params(d, n1, n2, k, r, T=T, seed=SEED + i, prec=prec, b_is_a=same)
    out = [torch.empty(n1, r, dtype=torch.float64, device=DEV), torch.empty(n2, r, dtype=torch.float64, device=DEV),
           torch.empty(r, dtype=torch.float64, device=DEV)]
    return dict(p=p, A=Ad, B=None if same else Bd, Ah=A, Bh=None if same else B, out=out)


def _alone(api, jobs):
    ctx = api.Context(0)
    res = []
    for j in jobs:
        U, V, s = [torch.empty_like(t) for t in j["out"]]
        ctx.smp_solve(j["p"], j["A"], j["B"], U, V, s)
        torch.cuda.synchronize()
        res.append((U, V, s))
    return res


def test_server_results_identical_alone_and_in_the_mix(api):
    jobs = [_make(api, i, j) for i, j in enumerate(JOBS)]
    alone = _alone(api, jobs)
    srv = api.Server(0, workers=4)
    ids = [srv.submit(j["p"], j["A"], j["B"], *j["out"]) for j in jobs]
    res = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.close()
    log(f"stats {st}; run ms {[round(r['run_ms'], 2) for r in res]}")
    assert all(r["status"] == 0 for r in res)
    for j, (U, V, s) in zip(jobs, alone):
        for a, b in zip(j["out"], (U, V, s)):
            assert torch.equal(a, b)
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["max_running"] >= 2          # jobs overlapped on the device
    assert len({r["worker"] for r in res}) >= 2


def test_budget_serialises_admission(api):
    jobs = [_make(api, i, j) for i, j in enumerate(JOBS[:5])]
    alone = _alone(api, jobs)
    srv = api.Server(0, workers=4, hbm_budget=1)    # every job exceeds it: one at a time
    ids = [srv.submit(j["p"], j["A"], j["B"], *j["out"]) for j in jobs]
    res = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in res)
    assert st["max_running"] == 1
    for j, (U, V, s) in zip(jobs, alone):
        assert torch.equal(j["out"][0], U) and torch.equal(j["out"][2], s)


def test_continuous_admission(api):
    """Jobs submitted while others run start before the earlier ones finish
    (the loop keeps running and admits as workers free up)."""
    jobs = [_make(api, i, JOBS[8]) for i in range(6)]
    srv = api.Server(0, workers=2)
    ids = [srv.submit(j["p"], j["A"], j["B"], *j["out"]) for j in jobs[:2]]
    ids += [srv.submit(j["p"], j["A"], j["B"], *j["out"]) for j in jobs[2:]]
    res = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in res)
    assert st["max_running"] == 2
    # later jobs queued behind the first two
    assert max(r["queue_ms"] for r in res[2:]) > 0.0


def test_server_rejects_invalid_job_and_keeps_serving(api):
    good = _make(api, 0, JOBS[0])
    srv = api.Server(0, workers=2)
    bad = api.make_params(100, 20, 20, 8, 25)         # r > n
    U = torch.empty(20, 25, dtype=torch.float64, device=DEV)
    A = torch.zeros(100, 20, device=DEV)
    with pytest.raises(api.SmpError) as e:
        srv.submit(bad, A, A, U, U)
    assert e.value.status == 1
    jid = srv.submit(good["p"], good["A"], good["B"], *good["out"])
    assert srv.wait(jid)["status"] == 0
    with pytest.raises(api.SmpError):
        srv.wait(jid)                                   # already waited
    srv.close()


def test_solve_batch_matches_oracle(api):
    cases = [(2000, 200, 200, 50, 5, 10, False), (1037, 77, 131, 37, 3, 8, False), (3000, 150, 150, 80, 4, 10, True)]
    jobs = []
    for i, (d, n1, n2, k, r, T, same) in enumerate(cases):
        A, B, Ad, Bd = latent(d, n1, n2, R=r, seed=SEED + i, same=same)
        p = api.make_params(d, n1, n2, k, r, T=T, seed=SEED, b_is_a=same, init_iters=40)
        jobs.append(dict(p=p, A=Ad, B=None if same else Bd, Ah=A.numpy(), Bh=None if same else B.numpy(),
                         U=torch.empty(n1, r, dtype=torch.float64, device=DEV),
                         V=torch.empty(n2, r, dtype=torch.float64, device=DEV),
                         sigma=torch.empty(r, dtype=torch.float64, device=DEV), r=r, k=k, T=T))
    st, res = api.solve_batch(jobs, workers=3)
    assert st == 0 and all(r["status"] == 0 for r in res)
    for j in jobs:
        ref = oso.smp_pca(j["Ah"], j["Bh"], j["r"], j["k"], j["p"].m, j["T"], SEED)
        M = oev.product(j["Ah"], j["Bh"])
        e_gpu = oev.relative_error(M, j["U"].cpu().numpy(), j["sigma"].cpu().numpy(), j["V"].cpu().numpy())
        e_ora = oev.relative_error(M, ref["Uc"], ref["sigma"], ref["Vc"])
        log(f"  batch job e_gpu={e_gpu:.6e} e_oracle={e_ora:.6e}")
        assert abs(e_gpu - e_ora) <= 1e-4 * e_ora + 1e-6


def test_non_finite_input_fails_that_job_only(api):
    """A NaN in one job's input: smp_solve returns SMP_ERR_NUMERIC with the
    outputs untouched, and inside a server mix that job fails with the same
    status while every other job is bit-identical to its solve alone."""
    jobs = [_make(api, i, j) for i, j in enumerate(JOBS[:6])]
    bad = 2
    jobs[bad]["A"][17, 5] = float("nan")
    alone = _alone(api, [j for i, j in enumerate(jobs) if i != bad])
    ctx = api.Context(0)
    U, V, s = [torch.full_like(t, 7.0) for t in jobs[bad]["out"]]
    with pytest.raises(api.SmpError) as e:
        ctx.smp_solve(jobs[bad]["p"], jobs[bad]["A"], jobs[bad]["B"], U, V, s)
    assert e.value.status == api.SMP_ERR_NUMERIC
    assert torch.all(U == 7.0) and torch.all(V == 7.0) and torch.all(s == 7.0)
    srv = api.Server(0, workers=3)
    ids = [srv.submit(j["p"], j["A"], j["B"], *j["out"]) for j in jobs]
    res = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.close()
    log(f"statuses {[r['status'] for r in res]}")
    assert res[bad]["status"] == api.SMP_ERR_NUMERIC and "non-finite" in res[bad]["error"]
    assert st["failed"] == 1 and st["completed"] == len(jobs)
    others = [j for i, j in enumerate(jobs) if i != bad]
    for j, (U, V, s) in zip(others, alone):
        assert all(torch.equal(a, b) for a, b in zip(j["out"], (U, V, s)))
    assert all(r["status"] == 0 for i, r in enumerate(res) if i != bad)


def test_try_submit_refuses_while_busy(api):
    """smp_server_try_submit answers SMP_ERR_BUSY (nothing queued) while the
    only worker runs a job, and admits the same job once the worker is free."""
    long_job = dict(p=api.make_params(100_000, 1024, 1024, 400, 10, T=10, seed=SEED), out=None)
    A = torch.randn(100_000, 1024, device=DEV)
    B = torch.randn(100_000, 1024, device=DEV)
    outs = [torch.empty(1024, 10, dtype=torch.float64, device=DEV), torch.empty(1024, 10, dtype=torch.float64, device=DEV),
            torch.empty(10, dtype=torch.float64, device=DEV)]
    small = _make(api, 0, JOBS[0])
    srv = api.Server(0, workers=1)
    jid = srv.submit(long_job["p"], A, B, *outs)          # several ms of work on the one worker
    assert srv.try_submit(small["p"], small["A"], small["B"], *small["out"]) is None
    assert srv.wait(jid)["status"] == 0
    jid2 = srv.try_submit(small["p"], small["A"], small["B"], *small["out"])
    assert jid2 is not None and srv.wait(jid2)["status"] == 0
    st = srv.stats()
    srv.close()
    assert st["refused"] == 1 and st["submitted"] == 2


def test_budget_bounds_memory_in_use(api):
    """With a finite budget the memory in use at every admission (retained
    worker workspace plus the running jobs' inputs and outputs) stays within
    it, and jobs still overlap."""
    jobs = [_make(api, i, JOBS[8]) for i in range(8)]
    p0 = jobs[0]["p"]
    io = 4 * p0.d * (p0.n1 + p0.n2) + 8 * (p0.n1 + p0.n2 + 1) * p0.r
    budget = int(2.5 * (api.smp_workspace_size(p0) + io))
    alone = _alone(api, jobs)
    srv = api.Server(0, workers=4, hbm_budget=budget)
    ids = [srv.submit(j["p"], j["A"], j["B"], *j["out"]) for j in jobs]
    res = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.close()
    log(f"budget {budget} stats {st}")
    assert all(r["status"] == 0 for r in res)
    assert 0 < st["max_budget_in_use"] <= budget
    assert 2 <= st["max_running"] <= 3
    for j, (U, V, s) in zip(jobs, alone):
        assert torch.equal(j["out"][0], U) and torch.equal(j["out"][2], s)


@pytest.mark.parametrize("graph", [True, False])
def test_batch_group_identical_to_each_job_alone(api, graph):
    """smp_solve_batch_group (steps 2-4 on worker threads, WAltMin for all jobs
    grouped) gives every job the bits of smp_solve, A = B and SPLIT jobs
    included."""
    jobs = [_make(api, i, j) for i, j in enumerate(JOBS)]
    d, n1, n2, k, r, T = 3000, 150, 110, 60, 5, 6
    A, B, Ad, Bd = latent(d, n1, n2, R=3, seed=SEED + 999)
    p = api.make_params(d, n1, n2, k, r, T=T, seed=SEED + 998, omega_mode=api.SMP_OMEGA_SPLIT)
    jobs.append(dict(p=p, A=Ad, B=Bd, out=[torch.empty(n1, r, dtype=torch.float64, device=DEV),
                                          torch.empty(n2, r, dtype=torch.float64, device=DEV),
                                          torch.empty(r, dtype=torch.float64, device=DEV)]))
    alone = _alone(api, jobs)
    batch = [dict(p=j["p"], A=j["A"], B=j["B"], U=j["out"][0], V=j["out"][1], sigma=j["out"][2]) for j in jobs]
    st, res = api.solve_batch_group(batch, workers=3, graph=graph)
    log(f"batch group: status {st}; workers {sorted({x['worker'] for x in res})}")
    assert st == 0 and all(x["status"] == 0 for x in res)
    for i, (j, ref) in enumerate(zip(jobs, alone)):
        for a, b in zip(j["out"], ref):
            assert torch.equal(a, b), f"job {i}"

"""The allocation-free estimate entry point (smp_estimate_noalloc: its
scratch in a file-scope device array) against smp_estimate (library
workspace) through the C-ABI: bit-identical estimates on the same inputs,
on two calls in a row, the second with a smaller grid, on the dense-tile and
the gather paths of Eq. (2); sizes beyond its limit are refused before any
launch."""

import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_common import DEV, SEED, log
from oracle import sample as osa

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def api():
    from paper_1610_06656_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def _inputs(n1, n2, k, m, seed):
    g = torch.Generator().manual_seed(seed)
    At = torch.randn(n1, k, generator=g)
    Bt = torch.randn(n2, k, generator=g)
    na2 = (torch.rand(n1, generator=g) * 5).float()
    nb2 = (torch.rand(n2, generator=g) * 5).float()
    na2[3] = 0.0                                         # a zero data norm: M~ = 0 on its row
    om = osa.sample(na2.double().numpy(), nb2.double().numpy(), m, SEED)
    return At.to(DEV), Bt.to(DEV), na2.to(DEV), nb2.to(DEV), om


def _omega(api, om, n1, n2):
    from gpu_common import omega_from_oracle
    o, _ = omega_from_oracle(om, n1, n2)
    return o


@pytest.mark.parametrize("n1,n2,k,m", [(700, 600, 96, 40000.0),     # dense: 64 x 64 MFMA tiles
                                       (1500, 900, 40, 3000.0)])     # sparse: gathers
def test_noalloc_estimate_matches_workspace_estimate_twice(api, ctx, n1, n2, k, m):
    for call, (a, b, kk, mm) in enumerate([(n1, n2, k, m), (n1 // 3, n2 // 2, k // 2, m / 8)]):
        log(f"noalloc estimate call {call}: n1={a} n2={b} k={kk} m={mm}")
        At, Bt, na2, nb2, om = _inputs(a, b, kk, mm, 11 + call)
        p = api.make_params(100, a, b, kk, 2, m=mm)
        o_ws = _omega(api, om, a, b)
        o_na = _omega(api, om, a, b)
        ctx.smp_estimate(p, At, Bt, na2, nb2, o_ws)
        ctx.smp_estimate_noalloc(p, At, Bt, na2, nb2, o_na)
        torch.cuda.synchronize()
        nnz = om.nnz
        assert nnz > 0
        x, y = o_ws.mt_csr[:nnz].cpu().numpy(), o_na.mt_csr[:nnz].cpu().numpy()
        assert np.array_equal(x.view(np.uint64), y.view(np.uint64))
        x, y = o_ws.mt_csc[:nnz].cpu().numpy(), o_na.mt_csc[:nnz].cpu().numpy()
        assert np.array_equal(x.view(np.uint64), y.view(np.uint64))
        assert np.any(x != 0.0)


def test_noalloc_estimate_a_equals_b(api, ctx):
    n = 300
    At, _, na2, _, om = _inputs(n, n, 64, 20000.0, 5)
    p = api.make_params(100, n, n, 64, 2, m=20000.0)
    om = osa.sample(na2.double().cpu().numpy(), na2.double().cpu().numpy(), 20000.0, SEED)
    o_ws, o_na = _omega(api, om, n, n), _omega(api, om, n, n)
    ctx.smp_estimate(p, At, At, na2, na2, o_ws)
    ctx.smp_estimate_noalloc(p, At, At, na2, na2, o_na)
    torch.cuda.synchronize()
    assert torch.equal(o_ws.mt_csr[:om.nnz], o_na.mt_csr[:om.nnz])
    assert torch.equal(o_ws.mt_csc[:om.nnz], o_na.mt_csc[:om.nnz])


def test_noalloc_estimate_refuses_grids_beyond_its_limit(api, ctx):
    from paper_1610_06656_amd.api import Omega
    n1, n2 = 600_000, 500_000                          # n1 + n2 > 2^20
    p = api.make_params(100, n1, n2, 8, 2, m=1000.0)
    o = Omega(n1, n2, 1, DEV)
    t = torch.zeros(8, device=DEV)
    with pytest.raises(api.SmpError) as e:
        ctx.smp_estimate_noalloc(p, t, t, t, t, o)
    assert e.value.status == 5 and "limit" in str(e.value)

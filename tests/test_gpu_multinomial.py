"""GPU parity of the row-wise multinomial sampler (Appendix D, "Sampling";
SMP_SAMPLE_MULTINOMIAL) against the oracle's definition
(oracle.multinomial): given the same FP32 squared norms, the sampled entries,
their weights w = N_ij / q_ij, the CSC listing and the SPLIT subsets are
identical bit for bit (integer CDF, exact 64 x 64-bit products, deterministic
sort). End to end, the solve with this sampler matches the oracle's error."""

import numpy as np
import pytest
import torch

import smp_inputs
from conftest import gpu_available
from gpu_common import DEV, SEED, latent, log, omega_to_host
from oracle import evaluate as oev
from oracle import multinomial as omn
from oracle import solve as oso

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def api():
    from paper_1610_06656_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def _norm_inputs(n1, n2, seed, zero_a=(), zero_b=(), heavy=False):
    rng = np.random.default_rng(seed)
    na2 = (rng.standard_normal(n1) ** 2 * np.arange(1, n1 + 1) ** -0.8).astype(np.float32)
    nb2 = (rng.standard_normal(n2) ** 2 * np.arange(1, n2 + 1) ** -0.5).astype(np.float32)
    na2[list(zero_a)] = 0
    nb2[list(zero_b)] = 0
    if heavy:
        nb2[1] = 1e4 * nb2.max()          # one column takes half of every row's draws
    return na2, nb2


CASES = {
    "c1_default_m": dict(n1=200, n2=200, m=None, r=5),
    "ragged": dict(n1=77, n2=131, m=500.0, r=3),
    "dense_over_m": dict(n1=40, n2=45, m=5e4, r=2),             # many repeats per entry
    "zero_norms": dict(n1=64, n2=66, m=None, r=4, zero_a=(0, 5), zero_b=(3,)),
    "heavy_column": dict(n1=300, n2=257, m=None, r=4, heavy=True),
    "split_T3": dict(n1=150, n2=90, m=None, r=4, T=3, split=True),
    "wide": dict(n1=1000, n2=4097, m=None, r=10),
    "tall": dict(n1=5000, n2=3, m=None, r=2),
    "one_by_one": dict(n1=1, n2=1, m=7.5, r=1),
    "empty": dict(n1=50, n2=60, m=1e-6, r=2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_multinomial_sample_bit_exact(api, ctx, name):
    c = CASES[name]
    n1, n2, r = c["n1"], c["n2"], c["r"]
    T = c.get("T", 10)
    split = c.get("split", False)
    log(f"multinomial sample {name}")
    na2, nb2 = _norm_inputs(n1, n2, 3, c.get("zero_a", ()), c.get("zero_b", ()), c.get("heavy", False))
    p = api.make_params(100, n1, n2, 8, r, T=T, m=c["m"], omega_mode=1 if split else 0, sampler="multinomial")
    ref = omn.sample(na2.astype(np.float64), nb2.astype(np.float64), p.m, p.seed, T=T, split=split)
    from paper_1610_06656_amd.api import Omega
    om = Omega(n1, n2, max(ref.nnz, 1), DEV, split=split)
    nnz = ctx.smp_sample(p, torch.from_numpy(na2).to(DEV), torch.from_numpy(nb2).to(DEV), om)
    torch.cuda.synchronize()
    log(f"  |Omega| {nnz} draws {int(ref.row_draws.sum())} max multiplicity {int(ref.count.max()) if ref.nnz else 0}")
    assert nnz == ref.nnz
    assert (ref.nnz == 0) == (name == "empty")
    h = omega_to_host(om)
    assert np.array_equal(h["rows"], ref.rows) and np.array_equal(h["cols"], ref.cols)
    assert np.array_equal(h["w"].view(np.uint64), ref.w.view(np.uint64))      # bitwise
    perm = np.lexsort((ref.rows, ref.cols))
    assert np.array_equal(h["csc_cols"], ref.cols[perm]) and np.array_equal(h["csc_rows"], ref.rows[perm])
    assert np.array_equal(h["csc_w"].view(np.uint64), ref.w[perm].view(np.uint64))
    if split:
        assert np.array_equal(h["sub"], ref.subset) and np.array_equal(h["csc_sub"], ref.subset[perm])


def test_multinomial_capacity_error_reports_size(api, ctx):
    na2, nb2 = _norm_inputs(50, 60, 1)
    p = api.make_params(100, 50, 60, 8, 3, m=5000.0, sampler="multinomial")
    ref = omn.sample(na2.astype(np.float64), nb2.astype(np.float64), p.m, p.seed)
    from paper_1610_06656_amd.api import Omega
    om = Omega(50, 60, 10, DEV)
    with pytest.raises(api.SmpError) as e:
        ctx.smp_sample(p, torch.from_numpy(na2).to(DEV), torch.from_numpy(nb2).to(DEV), om)
    assert e.value.status == 5 and om.nnz == ref.nnz


def test_multinomial_large_grid_sampled_rows(api, ctx):
    """n1 = n2 = 30,000 (9 x 10^8 grid entries, which the one-coin-per-entry
    sampler would visit; the draws are at most m + n1, m = 6.2 x 10^6): the
    whole listing against the oracle's."""
    n1 = n2 = 30_000
    r = 5
    na2, nb2 = _norm_inputs(n1, n2, 5)
    p = api.make_params(100, n1, n2, 8, r, m=None, sampler="multinomial")
    ref = omn.sample(na2.astype(np.float64), nb2.astype(np.float64), p.m, p.seed)
    from paper_1610_06656_amd.api import Omega
    om = Omega(n1, n2, ref.nnz, DEV)
    nnz = ctx.smp_sample(p, torch.from_numpy(na2).to(DEV), torch.from_numpy(nb2).to(DEV), om)
    torch.cuda.synchronize()
    log(f"  |Omega| {nnz} of {n1 * n2} entries, m = {p.m:.0f}")
    assert nnz == ref.nnz
    h = omega_to_host(om)
    assert np.array_equal(h["rows"], ref.rows) and np.array_equal(h["cols"], ref.cols)
    assert np.array_equal(h["w"].view(np.uint64), ref.w.view(np.uint64))
    assert np.array_equal(om.col_ptr.cpu().numpy(),
                          np.concatenate([[0], np.cumsum(np.bincount(ref.cols, minlength=n2))]))


def test_multinomial_solve_matches_oracle(api, ctx):
    """Alg. 1 end to end with the Appendix D sampler on the small workload
    (d = 2,000, n = 200, k = 50, r = 5): the GPU's spectral error within
    1e-4 (relative) of the oracle's, and within a factor of 2 of the binomial
    sampler's (Appendix D)."""
    c = smp_inputs.CONFIGS["c1_small"]
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=c["R"], sigma=c["sigma"], alpha=c["alpha"])
    M = oev.product(A.numpy(), B.numpy())
    errs = {}
    for sampler in ("multinomial", "binomial"):
        p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], init_iters=40, sampler=sampler)
        U = torch.empty(c["n1"], c["r"], dtype=torch.float64, device=DEV)
        V = torch.empty(c["n2"], c["r"], dtype=torch.float64, device=DEV)
        s = torch.empty(c["r"], dtype=torch.float64, device=DEV)
        ctx.smp_solve(p, Ad, Bd, U, V, s)
        torch.cuda.synchronize()
        errs[sampler] = oev.relative_error(M, U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy())
    ref = oso.smp_pca(A.numpy(), B.numpy(), c["r"], c["k"], p.m, c["T"], SEED, sampler="multinomial")
    e_ora = oev.relative_error(M, ref["Uc"], ref["sigma"], ref["Vc"])
    log(f"  multinomial gpu {errs['multinomial']:.6e} oracle {e_ora:.6e} binomial gpu {errs['binomial']:.6e}")
    assert abs(errs["multinomial"] - e_ora) <= 1e-4 * e_ora
    assert errs["multinomial"] <= 2.0 * errs["binomial"]

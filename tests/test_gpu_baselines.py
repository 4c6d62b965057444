"""GPU parity of the comparison methods (Section 4) against the oracle's
definitions (oracle.baselines):

  * SVD(A~^T B~): the GPU's top-r SVD of its FP32 sketches against the exact
    SVD of the oracle's FP64 sketches of the same matrices (same Pi): the
    rank-r products agree to 1e-5 (the sketches differ by ~1e-6 per column;
    40 subspace rounds), the spectral errors to 1e-4;
  * LELA: column norms against FP64 sums (1e-6), exact entries on a sample
    against the FP64 product (FP32 GEMM chunks of 65,536 rows: 1e-5), and the
    whole method's spectral error within 1e-4 of the oracle's.
"""

import numpy as np
import pytest
import torch

import smp_inputs
from conftest import gpu_available
from gpu_common import DEV, SEED, latent, log, omega_from_oracle, product
from oracle import baselines as obl
from oracle import evaluate as oev
from oracle import sample as osa
from oracle import solve as oso

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def api():
    from paper_1610_06656_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


CASES = {
    "c1": dict(d=2000, n1=200, n2=200, k=50, r=5),
    "ragged": dict(d=1037, n1=77, n2=131, k=37, r=3),
    "wide_k": dict(d=3000, n1=300, n2=260, k=400, r=10),
}


def _out(n1, n2, r):
    return (torch.empty(n1, r, dtype=torch.float64, device=DEV), torch.empty(n2, r, dtype=torch.float64, device=DEV),
            torch.empty(r, dtype=torch.float64, device=DEV))


@pytest.mark.parametrize("name", list(CASES))
def test_svd_of_sketch_product_matches_oracle(api, ctx, name):
    c = CASES[name]
    log(f"svd(A~^T B~) {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=min(5, c["n1"], c["n2"]))
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], init_iters=40)
    U, V, s = _out(c["n1"], c["n2"], c["r"])
    ctx.smp_solve_svd_sketch(p, Ad, Bd, U, V, s)
    torch.cuda.synchronize()
    Ug, sg, Vg = U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy()
    Uo, so, Vo = obl.svd_of_sketch_product(A.numpy(), B.numpy(), c["r"], c["k"], SEED)
    X, Xo = product(Ug, sg, Vg), product(Uo, so, Vo)
    rel = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    M = oev.product(A.numpy(), B.numpy())
    e, eo = oev.relative_error(M, Ug, sg, Vg), oev.relative_error(M, Uo, so, Vo)
    log(f"  product rel diff {rel:.2e}; error gpu {e:.6e} oracle {eo:.6e}")
    assert rel < 1e-5
    assert abs(e - eo) <= 1e-4 * eo
    assert np.allclose(Ug.T @ Ug, np.eye(c["r"]), atol=1e-10) and np.allclose(Vg.T @ Vg, np.eye(c["r"]), atol=1e-10)
    assert np.all(np.diff(sg) <= 1e-12 * sg[0])


def test_column_norms_and_exact_entries(api, ctx):
    d, n1, n2 = 150_000, 120, 90                     # three 65,536-row GEMM chunks
    A, B, Ad, Bd = latent(d, n1, n2)
    p = api.make_params(d, n1, n2, 8, 3)
    na2 = torch.empty(n1, device=DEV)
    nb2 = torch.empty(n2, device=DEV)
    ctx.smp_column_norms(p, Ad, Bd, na2, nb2)
    om = osa.sample(na2.double().cpu().numpy(), nb2.double().cpu().numpy(), 4000.0, SEED)
    o, _ = omega_from_oracle(om, n1, n2)
    ctx.smp_exact_entries(p, Ad, Bd, o)
    torch.cuda.synchronize()
    ref_a = obl.column_norms2(A.numpy())
    assert np.allclose(na2.cpu().numpy(), ref_a, rtol=1e-6, atol=0)
    assert np.allclose(nb2.cpu().numpy(), obl.column_norms2(B.numpy()), rtol=1e-6, atol=0)
    M = oev.product(A.numpy(), B.numpy())
    ref = M[om.rows, om.cols]
    scale = np.sqrt(ref_a[om.rows] * obl.column_norms2(B.numpy())[om.cols])
    got = o.mt_csr[:om.nnz].cpu().numpy()
    log(f"  |Omega| {om.nnz}: max |diff| / (||A_i|| ||B_j||) {np.max(np.abs(got - ref) / scale):.2e}")
    assert np.max(np.abs(got - ref) / scale) < 1e-5
    perm = np.lexsort((om.rows, om.cols))
    assert np.array_equal(o.mt_csc[:om.nnz].cpu().numpy(), got[perm])


@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_lela_matches_oracle(api, ctx, name):
    c = CASES[name]
    log(f"lela {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=min(5, c["n1"], c["n2"]))
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=10, init_iters=40)
    U, V, s = _out(c["n1"], c["n2"], c["r"])
    ctx.smp_lela(p, Ad, Bd, U, V, s)
    torch.cuda.synchronize()
    M = oev.product(A.numpy(), B.numpy())
    e = oev.relative_error(M, U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy())
    ref = obl.lela(A.numpy(), B.numpy(), c["r"], p.m, 10, SEED)
    eo = oev.relative_error(M, ref["Uc"], ref["sigma"], ref["Vc"])
    log(f"  lela error gpu {e:.6e} oracle {eo:.6e}")
    assert abs(e - eo) <= 1e-4 * eo


def test_c2_size_methods_ordering(api, ctx):
    """At d = 200,000, n = 2,000, k = 400, r = 10: the oracle's best rank-r
    error <= LELA <= SMP-PCA (Table 1's ordering), and SVD(A~^T B~)'s error
    reported beside them."""
    c = smp_inputs.CONFIGS["c2_fp32"]
    Ad, Bd = smp_inputs.latent_pair(c["d"], c["n1"], c["n2"], c["R"], c["sigma"], c["alpha"], SEED, device=DEV)
    M = torch.zeros(c["n1"], c["n2"], dtype=torch.float64, device=DEV)
    for l0 in range(0, c["d"], 1 << 16):
        M += Ad[l0:l0 + (1 << 16)].double().T @ Bd[l0:l0 + (1 << 16)].double()
    sv = torch.linalg.svdvals(M)
    opt = (sv[c["r"]] / sv[0]).item()
    errs = {}
    for name in ("smp", "lela", "svd"):
        p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"])
        U, V, s = _out(c["n1"], c["n2"], c["r"])
        {"smp": ctx.smp_solve, "lela": ctx.smp_lela, "svd": ctx.smp_solve_svd_sketch}[name](p, Ad, Bd, U, V, s)
        torch.cuda.synchronize()
        E = M - (U * s[None, :]) @ V.T
        errs[name] = (torch.linalg.matrix_norm(E, 2) / sv[0]).item()
    log(f"  optimal {opt:.6f} lela {errs['lela']:.6f} smp-pca {errs['smp']:.6f} svd(A~^T B~) {errs['svd']:.6f}")
    assert opt <= errs["lela"] <= errs["smp"]

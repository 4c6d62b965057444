"""GPU parity, stage by stage: each HIP stage (through the C-ABI) against the
oracle on the same inputs.

Tolerances (derived from the arithmetic):
  Pi            FP32 Box-Muller vs FP64: |dZ| <= 1e-5 (a few FP32 ulps of |Z| <= 6)
  sketch        FP32 MFMA accumulation: ||dA~_i|| / ||A~_i|| <= 1e-5 per column
  norms         compensated FP32 sums: relative 1e-6
  sampling      bit-exact (same FP32 norms in, binary64 decision in a fixed order)
  estimate      FP64 dot of the same FP32 sketches: |dM~_ij| <= 1e-10 ||A_i|| ||B_j||
  WAltMin       FP64: ||dX||_F / ||X||_F <= 1e-6 for the product U V^T
"""

import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_common import DEV, SEED, fixed_FA, latent, log, omega_from_oracle, omega_to_host, product
from oracle import estimate as oes
from oracle import philox, gaussian
from oracle import sample as osa
from oracle import sketch as osk
from oracle import waltmin as owm

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def api():
    from paper_1610_06656_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


# ---------------------------------------------------------------- a1: Pi

@pytest.mark.parametrize("k,l0,nrows", [(50, 0, 300), (13, 1000, 257), (400, 199_000, 64), (7, 2**32 - 3, 10)])
def test_pi_fill_matches_oracle(api, ctx, k, l0, nrows):
    log(f"pi_fill k={k} l0={l0} nrows={nrows}")
    p = api.make_params(d=l0 + nrows, n1=1, n2=1, k=k, r=1, m=1.0)
    out = torch.empty(nrows, k, dtype=torch.float32, device=DEV)
    ctx.smp_pi_fill(p, l0, nrows, out)
    torch.cuda.synchronize()
    ref = osk.pi_block(p.seed, k, l0, l0 + nrows).T
    dz = (out.cpu().numpy().astype(np.float64) - ref) * np.sqrt(k)
    assert np.abs(dz).max() < 1e-5
    assert np.sqrt(np.mean(dz**2)) < 1e-6


# ---------------------------------------------------------------- a2/a3: sketch

SKETCH_CASES = {
    "c1": dict(d=2000, n1=200, n2=200, k=50),
    "ragged": dict(d=1037, n1=77, n2=131, k=37),
    "k400_tiles": dict(d=20000, n1=300, n2=520, k=400),
    "k1024_chunks": dict(d=4096, n1=129, n2=64, k=1024),
    "tiny": dict(d=3, n1=1, n2=5, k=1),
}


def _oracle_sketch(A, B, seed, k):
    At, Bt, na2, nb2 = osk.sketch(A.numpy(), None if B is None else B.numpy(), seed, k)
    return At, Bt, na2, nb2


def _col_rel(got_t, ref):
    """max over columns of ||got_i - ref_i|| / ||ref_i|| (got transposed n x k)."""
    g = got_t.T.astype(np.float64)
    num = np.linalg.norm(g - ref, axis=0)
    den = np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
    return float(np.max(num / den))


@pytest.mark.parametrize("name", list(SKETCH_CASES))
def test_sketch_parity(api, ctx, name):
    c = SKETCH_CASES[name]
    log(f"sketch {name} {c}")
    A, B, Ad, Bd = latent(c["d"], c["n1"], c["n2"], R=min(5, c["n1"], c["n2"]))
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], r=1)
    At = torch.empty(c["n1"], c["k"], device=DEV)
    Bt = torch.empty(c["n2"], c["k"], device=DEV)
    na2 = torch.empty(c["n1"], device=DEV)
    nb2 = torch.empty(c["n2"], device=DEV)
    ctx.smp_sketch(p, Ad, Bd, At, Bt, na2, nb2)
    torch.cuda.synchronize()
    oAt, oBt, ona2, onb2 = _oracle_sketch(A, B, p.seed, c["k"])
    assert _col_rel(At.cpu().numpy(), oAt) < 1e-5
    assert _col_rel(Bt.cpu().numpy(), oBt) < 1e-5
    assert np.allclose(na2.cpu().numpy(), ona2, rtol=1e-6, atol=0)
    assert np.allclose(nb2.cpu().numpy(), onb2, rtol=1e-6, atol=0)


def test_sketch_padded_leading_dimension_and_zero_column(api, ctx):
    d, n1, n2, k = 700, 45, 33, 21
    A, B, _, _ = latent(d, n1, n2)
    A[:, 7] = 0.0
    Afull = torch.zeros(d, n1 + 3)
    Afull[:, :n1] = A
    Ad = Afull.to(DEV)[:, :n1]                 # lda = n1 + 3 (odd): scalar load path
    Bd = B.to(DEV)
    p = api.make_params(d, n1, n2, k, r=1)
    At = torch.empty(n1, k, device=DEV)
    Bt = torch.empty(n2, k, device=DEV)
    na2 = torch.empty(n1, device=DEV)
    nb2 = torch.empty(n2, device=DEV)
    ctx.smp_sketch(p, Ad, Bd, At, Bt, na2, nb2)
    torch.cuda.synchronize()
    oAt, oBt, ona2, onb2 = _oracle_sketch(A, B, p.seed, k)
    assert np.all(At.cpu().numpy()[7] == 0.0) and na2.cpu().numpy()[7] == 0.0
    keep = np.arange(n1) != 7
    assert _col_rel(At.cpu().numpy()[keep], oAt[:, keep]) < 1e-5
    assert _col_rel(Bt.cpu().numpy(), oBt) < 1e-5


def test_sketch_b_is_a(api, ctx):
    d, n, k = 1500, 96, 40
    A, _, Ad, _ = latent(d, n, n, same=True)
    p = api.make_params(d, n, n, k, r=1, b_is_a=True)
    At = torch.empty(n, k, device=DEV)
    Bt = torch.empty(n, k, device=DEV)
    na2 = torch.empty(n, device=DEV)
    nb2 = torch.empty(n, device=DEV)
    ctx.smp_sketch(p, Ad, None, At, Bt, na2, nb2)
    torch.cuda.synchronize()
    oAt, _, ona2, _ = _oracle_sketch(A, None, p.seed, k)
    assert _col_rel(At.cpu().numpy(), oAt) < 1e-5
    assert torch.equal(At, Bt) and torch.equal(na2, nb2)


def test_sketch_streaming_push_any_order(api, ctx):
    """Rows pushed in blocks, out of order (the arbitrary-order streaming of
    Section 1), give the one-pass result."""
    d, n1, n2, k = 3000, 130, 70, 64
    A, B, Ad, Bd = latent(d, n1, n2)
    p = api.make_params(d, n1, n2, k, r=1)
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
    oAt, oBt, ona2, onb2 = _oracle_sketch(A, B, p.seed, k)
    assert _col_rel(At.cpu().numpy(), oAt) < 1e-5
    assert _col_rel(Bt.cpu().numpy(), oBt) < 1e-5
    assert np.allclose(na2.cpu().numpy(), ona2, rtol=1e-6)


# ---------------------------------------------------------------- a4: sampling

def _norm_inputs(n1, n2, seed, zero_a=(), zero_b=()):
    rng = np.random.default_rng(seed)
    na2 = (rng.standard_normal(n1) ** 2 * np.arange(1, n1 + 1) ** -0.8).astype(np.float32)
    nb2 = (rng.standard_normal(n2) ** 2 * np.arange(1, n2 + 1) ** -0.5).astype(np.float32)
    na2[list(zero_a)] = 0
    nb2[list(zero_b)] = 0
    return na2, nb2


SAMPLE_CASES = {
    "c1_default_m": dict(n1=200, n2=200, m=None, r=5),
    "ragged_small_m": dict(n1=77, n2=131, m=50.0, r=3),
    "all_sampled": dict(n1=40, n2=45, m=1e9, r=2),
    "zero_norms": dict(n1=64, n2=66, m=None, r=4, zero_a=(0, 5), zero_b=(3,)),
    "split_T3": dict(n1=150, n2=90, m=None, r=4, T=3, split=True),
    "wide": dict(n1=1000, n2=2047, m=None, r=10),
    "empty": dict(n1=50, n2=60, m=1e-6, r=2),          # no entry kept
}


@pytest.mark.parametrize("name", list(SAMPLE_CASES))
def test_sample_bit_exact(api, ctx, name):
    c = SAMPLE_CASES[name]
    log(f"sample {name}")
    n1, n2, r = c["n1"], c["n2"], c["r"]
    T = c.get("T", 10)
    split = c.get("split", False)
    na2, nb2 = _norm_inputs(n1, n2, 3, c.get("zero_a", ()), c.get("zero_b", ()))
    p = api.make_params(100, n1, n2, 8, r, T=T, m=c["m"], omega_mode=1 if split else 0)
    from paper_1610_06656_amd.api import Omega
    om = Omega(n1, n2, n1 * n2, DEV, split=split)
    nnz = ctx.smp_sample(p, torch.from_numpy(na2).to(DEV), torch.from_numpy(nb2).to(DEV), om)
    torch.cuda.synchronize()
    ref = osa.sample(na2.astype(np.float64), nb2.astype(np.float64), p.m, p.seed, T=T, split=split)
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


def test_sample_capacity_error_reports_size(api, ctx):
    na2, nb2 = _norm_inputs(50, 60, 1)
    p = api.make_params(100, 50, 60, 8, 3, m=1e9)
    from paper_1610_06656_amd.api import Omega
    om = Omega(50, 60, 10, DEV)
    with pytest.raises(api.SmpError) as e:
        ctx.smp_sample(p, torch.from_numpy(na2).to(DEV), torch.from_numpy(nb2).to(DEV), om)
    assert e.value.status == 5 and om.nnz == 50 * 60


# ---------------------------------------------------------------- a3/a5: estimate

@pytest.mark.parametrize("name,d,n1,n2,k,m", [("c1_tiles", 2000, 200, 200, 50, None),
                                             ("ragged_tiles", 900, 77, 131, 37, None),
                                             ("k400_tiles", 5000, 120, 90, 400, None),
                                             ("mixed_blocks", 1000, 600, 700, 40, 40000.0),
                                             ("sparse_gather", 1000, 600, 700, 40, 2000.0)])
def test_estimate_parity(api, ctx, name, d, n1, n2, k, m):
    """Dense grids take the 64 x 64 MFMA tile path, sparse grids (Omega below
    1/32 of the grid) the gather path; both must give the oracle's values.
    "mixed_blocks" covers about 8% of the grid, dense in the heavy leading
    rows and sparse elsewhere."""
    log(f"estimate {name}")
    A, B, _, _ = latent(d, n1, n2)
    oAt, oBt, ona2, onb2 = osk.sketch(A.numpy(), B.numpy(), SEED, k)
    At32 = np.ascontiguousarray(oAt.T, dtype=np.float32)      # same FP32 inputs both sides
    Bt32 = np.ascontiguousarray(oBt.T, dtype=np.float32)
    na32, nb32 = ona2.astype(np.float32), onb2.astype(np.float32)
    om = osa.sample(na32.astype(np.float64), nb32.astype(np.float64), m or api.default_m(n1, n2, 5), SEED)
    assert (om.nnz * 32 < n1 * n2) == name.startswith("sparse")
    ref = oes.estimate(At32.T.astype(np.float64), Bt32.T.astype(np.float64), na32.astype(np.float64),
                       nb32.astype(np.float64), om.rows, om.cols)
    o, perm = omega_from_oracle(om, n1, n2)
    p = api.make_params(d, n1, n2, k, 5)
    ctx.smp_estimate(p, torch.from_numpy(At32).to(DEV), torch.from_numpy(Bt32).to(DEV),
                     torch.from_numpy(na32).to(DEV), torch.from_numpy(nb32).to(DEV), o)
    torch.cuda.synchronize()
    h = omega_to_host(o)
    scale = np.sqrt(na32.astype(np.float64)[om.rows] * nb32.astype(np.float64)[om.cols])
    assert np.max(np.abs(h["mt"] - ref) / scale) < 1e-10
    assert np.array_equal(h["csc_mt"], h["mt"][perm])          # both listings carry identical bits


def test_estimate_a_equals_b_diagonal(api, ctx):
    d, n, k = 800, 60, 30
    A, _, _, _ = latent(d, n, n, same=True)
    oAt, _, ona2, _ = osk.sketch(A.numpy(), None, SEED, k)
    At32, na32 = np.ascontiguousarray(oAt.T, dtype=np.float32), ona2.astype(np.float32)
    om = osa.sample(na32.astype(np.float64), na32.astype(np.float64), 1e9, SEED)    # all entries
    o, _ = omega_from_oracle(om, n, n)
    p = api.make_params(d, n, n, k, 3)
    At_d = torch.from_numpy(At32).to(DEV)
    na_d = torch.from_numpy(na32).to(DEV)
    ctx.smp_estimate(p, At_d, At_d, na_d, na_d, o)
    torch.cuda.synchronize()
    h = omega_to_host(o)
    diag = h["rows"] == h["cols"]
    assert np.allclose(h["mt"][diag], na32.astype(np.float64)[h["rows"][diag]], rtol=1e-14)


# ---------------------------------------------------------------- a6-a8: WAltMin

WALTMIN_CASES = {
    "c1_T10": dict(d=2000, n=200, k=50, r=5, T=10),
    "c1_T0_init": dict(d=2000, n=200, k=50, r=5, T=0),
    "ragged_r3": dict(d=1200, n1=77, n2=131, k=60, r=3, T=6),
    "r20_tiles": dict(d=3000, n=160, k=200, r=20, T=5, R=20),
    "split": dict(d=2000, n=200, k=100, r=4, T=2, split=True, mscale=6.0),
    "r28_wide": dict(d=3000, n=220, k=240, r=28, T=4, R=28),   # p = 33 columns in the initial subspace
    # Gram columns past the first 16 summed on the VALU (r + 1 <= 25)
    "r17_rem": dict(d=3000, n1=150, n2=190, k=200, r=17, T=4, R=17),
    "r24_rem": dict(d=3000, n=210, k=240, r=24, T=4, R=24),
}


@pytest.mark.parametrize("name", list(WALTMIN_CASES))
def test_waltmin_parity(api, ctx, name):
    _waltmin_parity(api, ctx, name)


def _waltmin_parity(api, ctx, name):
    c = WALTMIN_CASES[name]
    log(f"waltmin {name}")
    n1 = c.get("n1", c.get("n"))
    n2 = c.get("n2", c.get("n"))
    r, T, k = c["r"], c["T"], c["k"]
    split = c.get("split", False)
    A, B, _, _ = latent(c["d"], n1, n2, R=c.get("R", 5))
    oAt, oBt, ona2, onb2 = osk.sketch(A.numpy(), B.numpy(), SEED, k)
    na32, nb32 = ona2.astype(np.float32), onb2.astype(np.float32)
    m = api.default_m(n1, n2, r) * c.get("mscale", 1.0)
    om = osa.sample(na32.astype(np.float64), nb32.astype(np.float64), m, SEED, T=T, split=split)
    mt = oes.estimate(oAt, oBt, ona2, onb2, om.rows, om.cols)
    ref = owm.waltmin(n1, n2, om.rows, om.cols, om.w, mt, r, T, na32.astype(np.float64), fixed_FA(na32),
                      subset=om.subset)
    X_ref = ref["U"] @ ref["V"].T
    o, _ = omega_from_oracle(om, n1, n2, mt=mt, split=split)
    p = api.make_params(c["d"], n1, n2, k, r, T=T, m=m, omega_mode=1 if split else 0, init_iters=40)
    U = torch.empty(n1, r, dtype=torch.float64, device=DEV)
    V = torch.empty(n2, r, dtype=torch.float64, device=DEV)
    s = torch.empty(r, dtype=torch.float64, device=DEV)
    ctx.smp_waltmin(p, o, torch.from_numpy(na32).to(DEV), U, V, s)
    torch.cuda.synchronize()
    Ug, sg, Vg = U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy()
    X = product(Ug, sg, Vg)
    rel = np.linalg.norm(X - X_ref) / np.linalg.norm(X_ref)
    log(f"  rel diff {rel:.3e}")
    assert rel < 1e-6
    assert np.allclose(Ug.T @ Ug, np.eye(r), atol=1e-10) and np.allclose(Vg.T @ Vg, np.eye(r), atol=1e-10)
    assert np.all(np.diff(sg) <= 1e-12 * sg[0])
    _, s_ref, _ = owm.canonical(ref["U"], ref["V"])
    assert np.allclose(sg, s_ref, rtol=1e-6)


@pytest.mark.parametrize("T", [0, 3])
def test_waltmin_trim_fires_like_the_oracle(api, ctx, T):
    """Alg. 2 step 6 on a crafted case where it fires: a spike M~_00 = 100
    on top of a rank-2 signal (30 a b^T + 10 c d^T, unit a, b, c, d) makes
    the first singular vector almost e_0, but ||A_0|| is tiny, so ||U0_0||
    exceeds 8 sqrt(r) ||A_0|| / ||A||_F and row 0 of U0 is zeroed. The
    trimmed U0 keeps rank r (singular values 1 and 0.011), so every later
    least-squares problem has one solution and the product does not depend
    on how the fixed factor is orthonormalised. (A spike alone would leave
    a zero column, and the solution would then depend on the basis chosen
    for it.) The GPU's trimmed initial factors (T = 0) and the iterates from
    them (T = 3) match the oracle's product, and row 0 of the T = 0 output is
    zero."""
    n1 = n2 = 20
    r = 2
    rng = np.random.default_rng(0)
    a, b, c, dd = (x / np.linalg.norm(x) for x in (rng.standard_normal(n1), rng.standard_normal(n2),
                                                   rng.standard_normal(n1), rng.standard_normal(n2)))
    M = 30.0 * np.outer(a, b) + 10.0 * np.outer(c, dd) + 0.01 * rng.standard_normal((n1, n2))
    M[0, 0] += 100.0
    rows, cols = [a.ravel() for a in np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")]
    w = np.ones(rows.size)
    na32 = np.ones(n1, dtype=np.float32)
    na32[0] = 1e-6
    ref = owm.waltmin(n1, n2, rows, cols, w, M.ravel(), r, T, na32.astype(np.float64), fixed_FA(na32))
    assert ref["trimmed"][0] and ref["trimmed"].sum() == 1
    X_ref = ref["U"] @ ref["V"].T

    class Om:   # the oracle's fully observed grid in the form omega_from_oracle takes
        pass
    om = Om()
    om.nnz, om.rows, om.cols, om.w, om.subset = rows.size, rows, cols, w, None
    o, _ = omega_from_oracle(om, n1, n2, mt=M.ravel())
    p = api.make_params(1000, n1, n2, 8, r, T=T, m=1e6, init_iters=40)
    U = torch.empty(n1, r, dtype=torch.float64, device=DEV)
    V = torch.empty(n2, r, dtype=torch.float64, device=DEV)
    s = torch.empty(r, dtype=torch.float64, device=DEV)
    ctx.smp_waltmin(p, o, torch.from_numpy(na32).to(DEV), U, V, s)
    torch.cuda.synchronize()
    X = product(U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy())
    rel = np.linalg.norm(X - X_ref) / np.linalg.norm(X_ref)
    log(f"  trim T={T}: rel diff {rel:.3e}, |X[0,:]| max {np.abs(X[0]).max():.3e}")
    assert rel < 1e-6
    if T == 0:
        assert np.all(X[0] == 0.0)
        assert abs(X[0, 0]) < 1.0 < abs(M[0, 0])      # the spike is gone

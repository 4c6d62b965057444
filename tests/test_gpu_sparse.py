"""GPU parity of the entry-wise sketch (smp_sketch_push_coo / _csr: matrices
given as entries in any order, Section 1; O(nnz k), Section 3) against the
oracle's definition (oracle.sparse: Pi formed for the rows that occur, each
entry adding v Pi[:, l] in FP64), and of the solve from the pushed sketches.

Tolerances (from the arithmetic):
  Gaussian FP32 / SRHT  per column ||dA~_i|| / ||A~_i|| <= 1e-5: FP32 products
          and sums over at most 512 entries per segment, then an FP32 sum over
          segments; the GPU's Box-Muller uses the hardware log2/sqrt/sin/cos
          (a few FP32 ulps from the FP64 draw), as in the dense FP32 pass;
  BF16    2e-4, the bar of the dense BF16 pass (FP32 draws rounded to bfloat16
          can land on the other side of a rounding midpoint than the FP64 draw);
  norms   1e-6 (FP64 sums of FP32 squares, stored as FP32);
  solve   spectral error within 1e-4 (relative) of the oracle's on the same
          matrices.
Results that are unique are compared bit for bit: the sketch of the same
entries in another order, and CSR against COO.
"""

import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_common import DEV, SEED, log
from oracle import evaluate as oev
from oracle import solve as oso
from oracle import sparse as osp
from smp_inputs import sparse as spin

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-5
TOL_BF16 = 2e-4


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


def _dev(e):
    rows, cols, vals = e
    return (torch.from_numpy(np.ascontiguousarray(rows, dtype=np.int64)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(cols, dtype=np.int32)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(vals, dtype=np.float32)).to(DEV))


def _random_entries(rng, d, n, nnz, long_cols=()):
    """nnz distinct pairs; columns in long_cols get `count` extra rows each."""
    key = rng.choice(d * n, size=nnz, replace=False)
    rows, cols = key // n, key % n
    extra_r, extra_c = [], []
    for c, count in long_cols:
        r = rng.choice(d, size=count, replace=False)
        r = r[~np.isin(r, rows[cols == c])]
        extra_r.append(r)
        extra_c.append(np.full(r.size, c))
    rows = np.concatenate([rows] + extra_r).astype(np.int64)
    cols = np.concatenate([cols] + extra_c).astype(np.int32)
    p = rng.permutation(rows.size)
    return rows[p], cols[p], rng.standard_normal(rows.size).astype(np.float32)


def _push(api, ctx, p, A, B, n1, n2, k, csr=False, chunks=1):
    st = ctx.smp_sketch_begin(p)
    try:
        for which, e in ((api.SMP_MAT_A, A), (api.SMP_MAT_B, B)):
            if e is None:
                continue
            nnz = len(e[0])
            for c0 in range(chunks):
                sl = slice(c0 * nnz // chunks, (c0 + 1) * nnz // chunks)
                part = tuple(x[sl] for x in e)
                if csr:
                    _push_csr(api, ctx, st, which, part, p.d)
                else:
                    ctx.smp_sketch_push_coo(st, which, *_dev(part))
        At = torch.empty(n1, k, device=DEV)
        Bt = torch.empty(n2, k, device=DEV)
        na2 = torch.empty(n1, device=DEV)
        nb2 = torch.empty(n2, device=DEV)
        ctx.smp_sketch_end(st, At, Bt, na2, nb2)
        torch.cuda.synchronize()
    finally:
        ctx.smp_sketch_free(st)
    return At.cpu().numpy(), Bt.cpu().numpy(), na2.cpu().numpy(), nb2.cpu().numpy()


def _push_csr(api, ctx, st, which, e, d):
    rows, cols, vals = e
    o = np.lexsort((cols, rows))          # CSR: by row; inside a row any order would do
    rows, cols, vals = rows[o], cols[o], vals[o]
    row0 = int(rows.min()) if rows.size else 0
    nrows = (int(rows.max()) + 1 - row0) if rows.size else 0
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows - row0, minlength=nrows))]).astype(np.int64)
    ctx.smp_sketch_push_csr(st, which, row0, torch.from_numpy(rp).to(DEV),
                            torch.from_numpy(cols.astype(np.int32)).to(DEV),
                            torch.from_numpy(vals.astype(np.float32)).to(DEV))


CASES = {
    # (d, n1, n2, k, nnz_a, nnz_b, long columns of A: (column, extra rows))
    "k37_ragged": dict(d=1037, n1=77, n2=131, k=37, na=3000, nb=5000, long=((5, 900),)),
    "k400_two_groups": dict(d=5000, n1=60, n2=40, k=400, na=9000, nb=4000, long=((0, 2000), (59, 513))),
    "k1500_q2": dict(d=3000, n1=20, n2=30, k=1500, na=1500, nb=2500, long=((7, 1100),)),
    "k4096_q4": dict(d=2000, n1=6, n2=5, k=4096, na=300, nb=200, long=((2, 600),)),
    "k1": dict(d=50, n1=3, n2=4, k=1, na=40, nb=60, long=()),
    "one_entry": dict(d=10, n1=1, n2=1, k=8, na=1, nb=1, long=()),
    "exactly_512": dict(d=4000, n1=2, n2=2, k=64, na=0, nb=3, long=((0, 512), (1, 1024))),
}


@pytest.mark.parametrize("name", list(CASES))
def test_coo_push_matches_oracle(api, ctx, name):
    c = CASES[name]
    log(f"coo push {name} {c}")
    rng = np.random.default_rng(17)
    A = _random_entries(rng, c["d"], c["n1"], c["na"], c["long"])
    B = _random_entries(rng, c["d"], c["n2"], c["nb"])
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], r=1, m=100.0)   # m: the sketch does not use it
    At, Bt, na2, nb2 = _push(api, ctx, p, A, B, c["n1"], c["n2"], c["k"])
    oA, oB, ona, onb = osp.sketch_pair(A, B, c["d"], c["n1"], c["n2"], p.seed, c["k"])
    ea, eb = _col_rel(At, oA), _col_rel(Bt, oB)
    log(f"  rel A {ea:.2e} B {eb:.2e}")
    assert ea <= TOL and eb <= TOL
    assert np.allclose(na2, ona, rtol=1e-6, atol=0) and np.allclose(nb2, onb, rtol=1e-6, atol=0)


def test_bag_of_words_bf16_and_srht(api, ctx):
    c = spin.SPARSE_CONFIGS["s1_small"]
    A, B = spin.sparse_pair(c, SEED)
    d, n1, n2, k = c["d"], c["n1"], c["n2"], c["k"]
    A = (A[0], A[1], (A[2] * np.float32(1.37)).astype(np.float32))    # values that bfloat16 rounds
    for kw, okw, tol in ((dict(prec=api.SMP_PREC_BF16), dict(fmt="bf16"), TOL_BF16),
                         (dict(sketch="srht"), dict(kind="srht"), TOL),
                         (dict(), dict(), TOL)):
        log(f"bag of words {kw}")
        p = api.make_params(d, n1, n2, k, r=1, **kw)
        At, Bt, na2, nb2 = _push(api, ctx, p, A, B, n1, n2, k)
        oA, oB, ona, onb = osp.sketch_pair(A, B, d, n1, n2, p.seed, k, **okw)
        ea, eb = _col_rel(At, oA), _col_rel(Bt, oB)
        log(f"  rel A {ea:.2e} B {eb:.2e}")
        assert ea <= tol and eb <= tol
        assert np.allclose(na2, ona, rtol=1e-6) and np.allclose(nb2, onb, rtol=1e-6)


def test_order_csr_and_split_pushes(api, ctx):
    """Another arrival order and the CSR form give the same bits; pushes that
    split the entries agree to FP32 rounding."""
    rng = np.random.default_rng(5)
    d, n1, n2, k = 3000, 40, 50, 100
    A = _random_entries(rng, d, n1, 6000, ((3, 1500),))
    B = _random_entries(rng, d, n2, 4000)
    p = api.make_params(d, n1, n2, k, r=1)
    ref = _push(api, ctx, p, A, B, n1, n2, k)
    q = rng.permutation(len(A[0]))
    shuffled = _push(api, ctx, p, tuple(x[q] for x in A), B, n1, n2, k)
    csr = _push(api, ctx, p, A, B, n1, n2, k, csr=True)
    for a, b, c in zip(ref, shuffled, csr):
        assert np.array_equal(a, b) and np.array_equal(a, c)
    split = _push(api, ctx, p, A, B, n1, n2, k, chunks=3)
    assert _col_rel(split[0], ref[0].T.astype(np.float64)) <= 1e-6
    assert _col_rel(split[1], ref[1].T.astype(np.float64)) <= 1e-6


def test_dense_rows_and_entries_mix(api, ctx):
    """Rows [0, h) pushed dense and the entries of rows [h, d) pushed as COO give
    the dense sketch of the whole matrix."""
    rng = np.random.default_rng(6)
    d, n1, n2, k, h = 2000, 30, 20, 64, 700
    A = _random_entries(rng, d, n1, 5000)
    B = _random_entries(rng, d, n2, 3000)
    Ad, Bd = spin.densify(A, d, n1), spin.densify(B, d, n2)
    p = api.make_params(d, n1, n2, k, r=1)
    st = ctx.smp_sketch_begin(p)
    try:
        ctx.smp_sketch_push(st, torch.from_numpy(Ad[:h]).to(DEV), torch.from_numpy(Bd[:h]).to(DEV), 0)
        for which, e in ((api.SMP_MAT_A, A), (api.SMP_MAT_B, B)):
            sel = e[0] >= h
            ctx.smp_sketch_push_coo(st, which, *_dev(tuple(x[sel] for x in e)))
        At = torch.empty(n1, k, device=DEV)
        Bt = torch.empty(n2, k, device=DEV)
        na2 = torch.empty(n1, device=DEV)
        nb2 = torch.empty(n2, device=DEV)
        ctx.smp_sketch_end(st, At, Bt, na2, nb2)
        torch.cuda.synchronize()
    finally:
        ctx.smp_sketch_free(st)
    oA, oB, ona, onb = osp.sketch_pair(A, B, d, n1, n2, p.seed, k)
    assert _col_rel(At.cpu().numpy(), oA) <= TOL and _col_rel(Bt.cpu().numpy(), oB) <= TOL
    assert np.allclose(na2.cpu().numpy(), ona, rtol=1e-6) and np.allclose(nb2.cpu().numpy(), onb, rtol=1e-6)


def test_b_is_a_entries(api, ctx):
    rng = np.random.default_rng(7)
    d, n, k = 1500, 45, 50
    A = _random_entries(rng, d, n, 4000, ((9, 800),))
    p = api.make_params(d, n, n, k, r=1, b_is_a=True)
    At, Bt, na2, nb2 = _push(api, ctx, p, A, None, n, n, k)
    oA, _, ona, _ = osp.sketch_pair(A, None, d, n, n, p.seed, k)
    assert _col_rel(At, oA) <= TOL and np.array_equal(At, Bt)
    assert np.allclose(na2, ona, rtol=1e-6) and np.array_equal(na2, nb2)


def test_bad_pushes_are_rejected_and_leave_the_state(api, ctx):
    rng = np.random.default_rng(8)
    d, n1, n2, k = 500, 10, 12, 16
    A = _random_entries(rng, d, n1, 400)
    B = _random_entries(rng, d, n2, 300)
    p = api.make_params(d, n1, n2, k, r=1)
    ref = _push(api, ctx, p, A, B, n1, n2, k)
    st = ctx.smp_sketch_begin(p)
    try:
        bad_row = (np.array([3, d], dtype=np.int64), np.array([0, 1], dtype=np.int32), np.ones(2, np.float32))
        bad_col = (np.array([3, 4], dtype=np.int64), np.array([0, n1], dtype=np.int32), np.ones(2, np.float32))
        neg = (np.array([-1], dtype=np.int64), np.array([0], dtype=np.int32), np.ones(1, np.float32))
        dup = (np.array([3, 4, 3], dtype=np.int64), np.array([1, 1, 1], dtype=np.int32), np.ones(3, np.float32))
        for e in (bad_row, bad_col, neg, dup):
            with pytest.raises(api.SmpError) as ei:
                ctx.smp_sketch_push_coo(st, api.SMP_MAT_A, *_dev(e))
            assert ei.value.status == api._lib.SMP_ERR_INVALID_ARG
        with pytest.raises(api.SmpError):     # row_ptr not ending at nnz
            ctx.smp_sketch_push_csr(st, api.SMP_MAT_A, 0, torch.tensor([0, 1, 5], dtype=torch.int64, device=DEV),
                                    torch.zeros(2, dtype=torch.int32, device=DEV), torch.ones(2, device=DEV))
        with pytest.raises(api.SmpError):     # decreasing row_ptr
            ctx.smp_sketch_push_csr(st, api.SMP_MAT_A, 0, torch.tensor([0, 2, 1, 2], dtype=torch.int64, device=DEV),
                                    torch.tensor([0, 1], dtype=torch.int32, device=DEV), torch.ones(2, device=DEV))
        with pytest.raises(api.SmpError):     # rows past d
            ctx.smp_sketch_push_csr(st, api.SMP_MAT_A, d - 1, torch.tensor([0, 1, 2], dtype=torch.int64, device=DEV),
                                    torch.zeros(2, dtype=torch.int32, device=DEV), torch.ones(2, device=DEV))
        with pytest.raises(api.SmpError):
            ctx.smp_sketch_push_coo(st, 2, *_dev(A))
        # the state is untouched: the valid pushes now give the reference bits
        ctx.smp_sketch_push_coo(st, api.SMP_MAT_A, *_dev(A))
        ctx.smp_sketch_push_coo(st, api.SMP_MAT_B, *_dev(B))
        ctx.smp_sketch_push_coo(st, api.SMP_MAT_B, *_dev(tuple(x[:0] for x in B)))   # empty push
        out = [torch.empty(n1, k, device=DEV), torch.empty(n2, k, device=DEV), torch.empty(n1, device=DEV),
               torch.empty(n2, device=DEV)]
        ctx.smp_sketch_end(st, *out)
        torch.cuda.synchronize()
        for a, b in zip(ref, out):
            assert np.array_equal(a, b.cpu().numpy())
        with pytest.raises(api.SmpError) as ei:
            ctx.smp_sketch_push_coo(st, api.SMP_MAT_A, *_dev(A))
        assert ei.value.status == api._lib.SMP_ERR_STATE
    finally:
        ctx.smp_sketch_free(st)
    for kw in (dict(prec=api.SMP_PREC_FP8), dict(b_is_a=True)):
        p2 = api.make_params(d, n1, n1, k, r=1, **kw)
        st = ctx.smp_sketch_begin(p2)
        try:
            with pytest.raises(api.SmpError):
                ctx.smp_sketch_push_coo(st, api.SMP_MAT_B if kw.get("b_is_a") else api.SMP_MAT_A, *_dev(A))
        finally:
            ctx.smp_sketch_free(st)


def test_solve_from_pushed_entries_matches_oracle(api, ctx):
    c = spin.SPARSE_CONFIGS["s1_small"]
    A, B = spin.sparse_pair(c, SEED)
    d, n1, n2, k, r, T = c["d"], c["n1"], c["n2"], c["k"], c["r"], c["T"]
    p = api.make_params(d, n1, n2, k, r, T=T, init_iters=40)
    At, Bt, na2, nb2 = (torch.from_numpy(x).to(DEV) for x in _push(api, ctx, p, A, B, n1, n2, k))
    U = torch.empty(n1, r, dtype=torch.float64, device=DEV)
    V = torch.empty(n2, r, dtype=torch.float64, device=DEV)
    s = torch.empty(r, dtype=torch.float64, device=DEV)
    ctx.smp_solve_sketched(p, At, Bt, na2, nb2, U, V, s)
    Ad, Bd = spin.densify(A, d, n1), spin.densify(B, d, n2)
    M = oev.product(Ad, Bd)
    e = oev.relative_error(M, U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy())
    ref = oso.smp_pca(Ad, Bd, r, k, p.m, T, SEED)
    eo = oev.relative_error(M, ref["Uc"], ref["sigma"], ref["Vc"])
    log(f"  sparse solve error gpu {e:.6e} oracle {eo:.6e}")
    assert abs(e - eo) <= 1e-4 * eo


def test_solve_sketched_equals_solve(api, ctx):
    """smp_solve_sketched on smp_sketch's outputs gives smp_solve's bits."""
    from gpu_common import latent
    A, B, Ad, Bd = latent(3000, 90, 70, R=4)
    d, n1, n2, k, r = 3000, 90, 70, 40, 4
    p = api.make_params(d, n1, n2, k, r, T=6)
    outs = []
    for mode in ("solve", "sketched"):
        U = torch.empty(n1, r, dtype=torch.float64, device=DEV)
        V = torch.empty(n2, r, dtype=torch.float64, device=DEV)
        s = torch.empty(r, dtype=torch.float64, device=DEV)
        if mode == "solve":
            ctx.smp_solve(p, Ad, Bd, U, V, s)
        else:
            At = torch.empty(n1, k, device=DEV)
            Bt = torch.empty(n2, k, device=DEV)
            na2 = torch.empty(n1, device=DEV)
            nb2 = torch.empty(n2, device=DEV)
            ctx.smp_sketch(p, Ad, Bd, At, Bt, na2, nb2)
            ctx.smp_solve_sketched(p, At, Bt, na2, nb2, U, V, s)
        outs.append([x.cpu().numpy() for x in (U, V, s)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_url_shape_full_size_against_the_dense_pass(api, ctx):
    """The URL-reputation shape at full size (d = 792,145, two sets of 10,000
    features, ~20 M entries each, k = 2,000): columns of a few hundred to a few
    thousand entries against the oracle one by one, and every column (the
    heaviest holds ~690,000 entries) against the GPU's dense FP32 pass on the
    densified matrix (itself held to the oracle by the dense parity tests)."""
    c = spin.SPARSE_CONFIGS["s3_url"]
    A, B = spin.sparse_pair(c, SEED)
    d, n1, n2, k = c["d"], c["n1"], c["n2"], c["k"]
    log(f"url shape: nnz A {len(A[0])} B {len(B[0])}")
    p = api.make_params(d, n1, n2, k, r=1)
    At, Bt, na2, nb2 = _push(api, ctx, p, A, B, n1, n2, k)
    cnt = np.bincount(A[1], minlength=n1)
    picks = [int(np.argmin(np.abs(cnt - t))) for t in (300, 1000, 3000)]
    for i in picks:
        sel = A[1] == i
        ref, rn = osp.sketch_entries(A[0][sel], np.zeros(sel.sum(), np.int32), A[2][sel], d, 1, p.seed, k)
        rel = np.linalg.norm(At[i].astype(np.float64) - ref[:, 0]) / np.linalg.norm(ref[:, 0])
        log(f"  column {i} ({cnt[i]} entries): rel {rel:.2e}")
        assert rel <= TOL and abs(na2[i] - rn[0]) <= 1e-6 * rn[0]
    # every column of A against the dense pass on the densified A (31.7 GB FP32)
    Ad = torch.zeros(d, n1, device=DEV)
    rows, cols, vals = _dev(A)
    Ad[rows, cols.long()] = vals
    del rows, cols, vals
    Dt = torch.empty(n1, k, device=DEV)
    dn = torch.empty(n1, device=DEV)
    pa = api.make_params(d, n1, n1, k, r=1, b_is_a=True)
    ctx.smp_sketch(pa, Ad, None, Dt, None, dn, None)
    torch.cuda.synchronize()
    del Ad
    torch.cuda.empty_cache()
    D = Dt.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(At.astype(np.float64) - D, axis=1) / np.linalg.norm(D, axis=1)
    log(f"  all columns vs dense pass: max rel {rel.max():.2e} (heaviest column {cnt.max()} entries)")
    assert rel.max() <= 2 * TOL
    assert np.allclose(na2, dn.cpu().numpy(), rtol=2e-6)

"""Shared helpers of the GPU parity tests: build inputs once, hand the same
values to the HIP path (through the C-ABI binding) and to the oracle."""

import numpy as np
import torch

import smp_inputs
from oracle import sample as osa

DEV = "cuda:0"
SEED = smp_inputs.SEED_BASE


def log(msg):
    print(msg, flush=True)


def latent(d, n1, n2, R=5, sigma=0.1, alpha=0.5, seed=SEED, same=False):
    """Inputs on the CPU generator (so small cases do not depend on the GPU's
    stream), returned as (A_cpu, B_cpu, A_dev, B_dev) FP32."""
    A, B = smp_inputs.latent_pair(d, n1, n2, R, sigma, alpha, seed, device="cpu", same=same)
    return A, B, A.to(DEV), (A.to(DEV) if same else B.to(DEV))


def omega_from_oracle(om, n1, n2, mt=None, split=False):
    """Device smp_omega arrays holding the oracle's sample (CSR order as drawn,
    CSC order by (column, row))."""
    from paper_1610_06656_amd.api import Omega
    nnz = om.nnz
    o = Omega(n1, n2, nnz, DEV, split=split)
    rows, cols = om.rows, om.cols
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n1))])
    perm = np.lexsort((rows, cols))
    cp = np.concatenate([[0], np.cumsum(np.bincount(cols, minlength=n2))])
    o.row_ptr.copy_(torch.from_numpy(rp.astype(np.int64)))
    o.col_ptr.copy_(torch.from_numpy(cp.astype(np.int64)))
    if nnz:
        o.col_idx[:nnz].copy_(torch.from_numpy(cols.astype(np.int32)))
        o.row_idx[:nnz].copy_(torch.from_numpy(rows[perm].astype(np.int32)))
        o.w_csr[:nnz].copy_(torch.from_numpy(om.w))
        o.w_csc[:nnz].copy_(torch.from_numpy(om.w[perm]))
        if mt is not None:
            o.mt_csr[:nnz].copy_(torch.from_numpy(mt))
            o.mt_csc[:nnz].copy_(torch.from_numpy(mt[perm]))
        if split:
            o.sub_csr[:nnz].copy_(torch.from_numpy(om.subset.astype(np.uint8)))
            o.sub_csc[:nnz].copy_(torch.from_numpy(om.subset[perm].astype(np.uint8)))
    o.nnz = nnz
    return o, perm


def omega_to_host(o):
    """(rows, cols, w, mt, sub) in CSR order and the CSC arrays, as numpy."""
    nnz = o.nnz
    rp = o.row_ptr.cpu().numpy()
    rows = np.repeat(np.arange(o.n1), np.diff(rp))
    cp = o.col_ptr.cpu().numpy()
    ccols = np.repeat(np.arange(o.n2), np.diff(cp))
    out = dict(rows=rows, cols=o.col_idx[:nnz].cpu().numpy().astype(np.int64),
               w=o.w_csr[:nnz].cpu().numpy(), mt=o.mt_csr[:nnz].cpu().numpy(),
               csc_cols=ccols, csc_rows=o.row_idx[:nnz].cpu().numpy().astype(np.int64),
               csc_w=o.w_csc[:nnz].cpu().numpy(), csc_mt=o.mt_csc[:nnz].cpu().numpy())
    if o.sub_csr is not None:
        out["sub"] = o.sub_csr[:nnz].cpu().numpy()
        out["csc_sub"] = o.sub_csc[:nnz].cpu().numpy()
    return out


def fixed_FA(na2_f32):
    return osa.fixed_order_sum(np.asarray(na2_f32, dtype=np.float64))


def product(U, s, V):
    return (U * s[None, :]) @ V.T

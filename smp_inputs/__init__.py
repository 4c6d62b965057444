"""Seeded synthetic inputs for SMP-PCA tests and benchmarks.

This module holds no arithmetic of the method. It only builds the d x n matrices
A and B that both the GPU path and the CPU oracle consume, so the two sides
always see the same FP32 values.

The paper's workloads are dense tall matrices with heavy-tailed column norms:
  * synthetic G D with G standard Gaussian and D_ii = 1/i (Section 4, datasets);
  * bag-of-words and URL feature matrices with d >> n (Table 1). Those datasets
    are not available here; the power-law column scaling below stands in for
    their skewed column norms.

Generator ("latent" family):
  Z (d x R), W_A, W_B (R x n), N_A, N_B (d x n), all i.i.d. N(0, 1) from a
  seeded torch.Generator on the requested device;
  A = (Z W_A + sigma N_A) diag((j+1)^-alpha),  B = (Z W_B + sigma N_B) diag((j+1)^-alpha).
The shared latent Z makes A^T B approximately rank R plus noise.

The random stream depends on the device (torch's CPU and GPU generators differ);
tests build A and B once and hand the same tensors to both sides.

Sparse inputs given as entries in arbitrary order (bag-of-words and URL-feature
shapes) come from ``smp_inputs.sparse``.
"""

import math

import torch

SEED_BASE = 161006656  # the arXiv number of the paper


def latent_pair(d, n1, n2, R, sigma, alpha, seed, device="cpu", same=False, chunk=1 << 16):
    """Return (A, B) as FP32 tensors of shape (d, n1) and (d, n2) on `device`.

    same=True returns (A, A) (the PCA case A = B). Rows are generated in chunks
    so that large d fits in memory without a d x n FP64 intermediate.
    """
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    WA = torch.randn(R, n1, generator=g, device=device, dtype=torch.float32)
    WB = WA if same else torch.randn(R, n2, generator=g, device=device, dtype=torch.float32)
    sa = torch.arange(1, n1 + 1, device=device, dtype=torch.float32).pow(-alpha)
    sb = torch.arange(1, n2 + 1, device=device, dtype=torch.float32).pow(-alpha)
    A = torch.empty(d, n1, device=device, dtype=torch.float32)
    B = A if same else torch.empty(d, n2, device=device, dtype=torch.float32)
    for l0 in range(0, d, chunk):
        l1 = min(d, l0 + chunk)
        Z = torch.randn(l1 - l0, R, generator=g, device=device, dtype=torch.float32)
        NA = torch.randn(l1 - l0, n1, generator=g, device=device, dtype=torch.float32)
        A[l0:l1] = (Z @ WA + sigma * NA) * sa
        if not same:
            NB = torch.randn(l1 - l0, n2, generator=g, device=device, dtype=torch.float32)
            B[l0:l1] = (Z @ WB + sigma * NB) * sb
    return A, B


def gd_pair(d, n1, n2, seed, device="cpu"):
    """The paper's synthetic family: A = G_A D, B = G_B D with G i.i.d. N(0,1)
    and D_ii = 1/i (Section 4, "Description of datasets")."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    A = torch.randn(d, n1, generator=g, device=device) / torch.arange(1, n1 + 1, device=device, dtype=torch.float32)
    B = torch.randn(d, n2, generator=g, device=device) / torch.arange(1, n2 + 1, device=device, dtype=torch.float32)
    return A, B


def cone_pair(d, n, theta, seed, device="cpu"):
    """Unit columns drawn from a cone of angle theta around a fixed unit x:
    y = +/-(x + t) normalised, t Gaussian with expected norm tan(theta/2)
    (Section 2, Figure 2 caption)."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    x = torch.randn(d, generator=g, device=device, dtype=torch.float64)
    x = x / x.norm()

    def draw():
        t = torch.randn(d, n, generator=g, device=device, dtype=torch.float64) * (math.tan(theta / 2) / math.sqrt(d))
        y = x[:, None] + t
        s = torch.where(torch.rand(n, generator=g, device=device) < 0.5, -1.0, 1.0).to(torch.float64)
        y = y * s[None, :]
        return (y / y.norm(dim=0, keepdim=True)).to(torch.float32)

    return draw(), draw()


# The workload shapes (rows of the benchmark/parity table). m = None means
# 4 n r ln n with n = max(n1, n2).
CONFIGS = {
    "c1_small": dict(d=2000, n1=200, n2=200, R=5, sigma=0.1, alpha=0.5, k=50, r=5, T=10),
    "c2_fp32": dict(d=200_000, n1=2000, n2=2000, R=10, sigma=0.1, alpha=0.5, k=400, r=10, T=10),
    "c3_precision": dict(d=1_000_000, n1=4096, n2=4096, R=20, sigma=0.05, alpha=0.7, k=1024, r=20, T=10),
}

# Job mixes for batching and serving: shapes and method parameters drawn per
# job (no arithmetic of the method). Each job reads the top-left d x n block
# of one of `pools` resident input pairs (generated at the largest shape with
# their own seeds), and has its own seed for Pi and the sampling coins.
BATCH = dict(jobs=512, d=(10_000, 200_000), n=(128, 2048), r=(5, 10, 20), k_over_r=(4, 20), R=10, sigma=0.1,
             alpha=0.5, T=10, pools=8)
SERVE = dict(rate_per_s=200.0, large_frac=0.05, large=dict(d=1_000_000, n=4096, r=20), R=20, sigma=0.05, alpha=0.7)


def job_mix(count, seed, large_frac=0.0):
    """`count` jobs as dicts (d, n, r, k, seed, pool, large) drawn as the
    batching mix: d uniform in [10k, 200k], n uniform in [128, 2048],
    r in {5, 10, 20}, k = r * uniform{4..20}; with probability large_frac a
    job is large (d = 1M, n = 4096, r = 20)."""
    rng = torch.Generator().manual_seed(int(seed))
    b = BATCH
    out = []
    for i in range(count):
        u = torch.rand(6, generator=rng).tolist()
        large = u[5] < large_frac
        if large:
            L = SERVE["large"]
            d, n, r = L["d"], L["n"], L["r"]
        else:
            d = int(b["d"][0] + u[0] * (b["d"][1] - b["d"][0]))
            n = int(b["n"][0] + u[1] * (b["n"][1] - b["n"][0]))
            r = b["r"][min(2, int(u[2] * 3))]
        k = r * int(b["k_over_r"][0] + u[3] * (b["k_over_r"][1] - b["k_over_r"][0] + 1))
        out.append(dict(d=d, n=n, r=r, k=min(k, 4096), seed=int(seed) * 1000003 + i,
                        pool=int(u[4] * b["pools"]) % b["pools"], large=large))
    return out

"""Writes tests/golden/c3_oracle.json: the oracle's end-to-end results on the
large precision workload (d = 10^6, n1 = n2 = 4096, latent rank 20, noise
0.05, column scale (j+1)^-0.7; k = 1024, r = 20, T = 10, m = 4 n r ln n),
which the oracle needs minutes for, so the GPU tests compare against stored
values instead of rerunning it.

    python tests/golden/make_c3_oracle.py

Calls only oracle/ and smp_inputs (the seeded input builder, CPU generator):
  * A^T B and A^T A in FP64 (oracle.evaluate.product, chunked over d), their
    best rank-r errors sigma_{r+1}/sigma_1 (Section 4, "Optimal");
  * Alg. 1 end to end (oracle.solve.smp_pca) with the FP64 sketch and with
    the BF16 and FP8 sketch definitions, and the A = B case (FP64 and BF16);
  * for each: the spectral error ||A^T B - U diag(s) V^T|| / ||A^T B||
    (Section 4's metric), |Omega|, and the wall time on this host.
The inputs are fingerprinted (FP64 sums over a strided subset of rows) so a
test can check that it rebuilt the same matrices.
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import smp_inputs  # noqa: E402
from oracle import evaluate, solve  # noqa: E402

OUT = os.path.join(HERE, "c3_oracle.json")


def fingerprint(X):
    """FP64 column sums of every 997th row of X (d x n): 4096 numbers that
    change if the generator's stream changes."""
    return np.asarray(X[::997], dtype=np.float64).sum(axis=0)


def main():
    c = smp_inputs.CONFIGS["c3_precision"]
    seed = smp_inputs.SEED_BASE
    from threadpoolctl import threadpool_info
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    t0 = time.perf_counter()
    A, B = smp_inputs.latent_pair(c["d"], c["n1"], c["n2"], c["R"], c["sigma"], c["alpha"], seed, device="cpu")
    A, B = A.numpy(), B.numpy()
    out = dict(config=c, seed=seed, m=solve.default_m(c["n1"], c["n2"], c["r"]), host_threads=int(threads),
               inputs_s=round(time.perf_counter() - t0, 1),
               fingerprint_A=fingerprint(A).tolist(), fingerprint_B=fingerprint(B).tolist(), runs={})
    print(f"inputs {out['inputs_s']} s", flush=True)

    for label, same in (("AB", False), ("AA", True)):
        t0 = time.perf_counter()
        M = evaluate.product(A, None if same else B)
        out[f"optimal_{label}"] = evaluate.optimal_error(M, c["r"])
        out[f"product_{label}_s"] = round(time.perf_counter() - t0, 1)
        print(f"product {label}: optimal {out[f'optimal_{label}']:.6e} ({out[f'product_{label}_s']} s)", flush=True)
        fmts = (None, "bf16", "fp8") if not same else (None, "bf16")
        for fmt in fmts:
            t0 = time.perf_counter()
            res = solve.smp_pca(A, None if same else B, c["r"], c["k"], out["m"], c["T"], seed, sketch_fmt=fmt)
            dt = time.perf_counter() - t0
            e = evaluate.relative_error(M, res["Uc"], res["sigma"], res["Vc"])
            key = f"{label}_{fmt or 'fp64'}"
            out["runs"][key] = dict(error=e, omega_nnz=int(res["omega"].nnz), sigma=res["sigma"].tolist(),
                                    oracle_s=round(dt, 1))
            print(f"{key}: error {e:.8e} |Omega| {res['omega'].nnz} ({dt:.1f} s)", flush=True)
            del res
        del M
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()

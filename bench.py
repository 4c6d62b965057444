"""Benchmark of the SMP-PCA hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload c3|c2|batch|serve|sparse] [--legs bf16,fp8,fp32,ab]
                    [--no-c2] [--no-mix]

A step is one smp_solve (Alg. 1 end to end: sketch pass, sampling, rescaled-JL
estimates, WAltMin, canonical form) with A and B already resident in HBM.

Default workload (one JSON line): the large precision workload,
d = 1,000,000, n1 = n2 = 4,096, k = 1,024, r = 20, T = 10, m = 4 n r ln n
(latent rank 20, noise 0.05, column scaling (j+1)^-0.7). `value` is input
bytes consumed per second, 4 d (n1+n2) / t, of the whole BF16-sketch solve
(sketch GEMM operands rounded to bfloat16, FP32 accumulation, FP64 WAltMin).
Beside it, at the same size: the FP8 E4M3 block-scaled sketch ("fp8"), the
plain FP32 sketch ("fp32"), the PCA case A = B ("ab", BF16) and the SRHT
sketch ("srht", FP32), each with its spectral error; the roofline of the BF16 sketch pass (MFMA-bound at this size)
with its HBM rate; the d = 200,000, n = 2,000, k = 400 workload ("c2", BF16
and FP32, and the paper's comparison methods LELA and SVD(A~^T B~) beside
SMP-PCA with their errors); the one-coin-per-entry and the row-wise
multinomial samplers ("sampler", n up to 100,000); sparse inputs pushed as
entries in random order ("sparse": the URL-reputation and NIPS-BW shapes,
Gaussian FP32 / BF16 and SRHT sketches, with the accumulation kernel against
its vector-ALU peak and the spectral errors); the batching mix (512 jobs)
and the Poisson serving mix ("batch", "serve", solves/s and p50/p99 latency,
BF16 vs FP32); and the FP64 CPU oracle's sketch pass timed on the host over a
stated number of rows.

--workload c2|batch|serve|sparse prints the single-workload lines instead.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sketch-pass GB/s + MFMA util; solves/s & p99 latency, BF16 vs FP32 plain"
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0   # dense
PEAK_FP8_MFMA_TFLOPS = 5000.0    # dense
PEAK_HBM_GBPS = 8000.0
C2 = dict(d=200_000, n1=2000, n2=2000, R=10, sigma=0.1, alpha=0.5, k=400, r=10, T=10)
C3 = dict(d=1_000_000, n1=4096, n2=4096, R=20, sigma=0.05, alpha=0.7, k=1024, r=20, T=10)
LEGS = ("bf16", "fp8", "fp32", "ab", "srht")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="rows of the CPU-oracle sketch sample (0: 200,000 at the large workload, all at c2)")
    ap.add_argument("--workload", choices=("c3", "c2", "batch", "serve", "sparse"), default="c3",
                    help="c3: the large precision workload with every leg (default); c2: d = 200,000 only; "
                         "batch: 512 jobs of the batching mix; serve: Poisson arrivals of the serving mix; "
                         "sparse: entry pushes of the sparse shapes only")
    ap.add_argument("--legs", default=",".join(LEGS), help="legs of the large workload to run (bf16,fp8,fp32,ab)")
    ap.add_argument("--no-c2", action="store_true", help="skip the d = 200,000 leg of the default line")
    ap.add_argument("--no-mix", action="store_true", help="skip the batching and serving legs of the default line")
    ap.add_argument("--no-sparse", action="store_true", help="skip the entry-push (sparse input) legs of the default line")
    ap.add_argument("--tune", action="store_true",
                    help="run smp_tune_sketch for the BF16, FP8 and A = B shapes of the large workload before the "
                         "timed legs (the legs then use the tuned launch shapes)")
    ap.add_argument("--no-errors", action="store_true", help="skip the spectral errors (profiling runs)")
    ap.add_argument("--workers", type=int, default=4, help="server worker threads (batch, serve)")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="arrival window of the serve workload")
    ap.add_argument("--serve-budget-gb", type=float, default=96.0,
                    help="HBM budget of the serve workload's server (GB of workspace, inputs and outputs of the "
                         "running jobs; 0: none)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of 2^30 bytes (the reference dispatch for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def recorded_traffic(name):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    runs (profiles/<name>.json), or None when the kernel's sources changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sha256"] else None


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
    return xs[i]


def _threads():
    from threadpoolctl import threadpool_info
    return int(max([t.get("num_threads", 1) for t in threadpool_info()] or [1]))


def cpu_baseline_pipeline(A, B, c, m, seed, rows):
    """The oracle as it stands (FP64 numpy) on a bounded sample of the same
    workload: the first `rows` rows of A and B, the full downstream pipeline."""
    from oracle import solve as osolve

    d_s = min(rows or c["d"], c["d"])
    a = A[:d_s].cpu().numpy()
    b = B[:d_s].cpu().numpy()
    t0 = time.perf_counter()
    osolve.smp_pca(a, b, c["r"], c["k"], m, c["T"], seed)
    dt = time.perf_counter() - t0
    gbytes = 4.0 * d_s * (c["n1"] + c["n2"]) / 1e9
    return {"value": gbytes / dt, "unit": "GB/s", "cores": _threads(), "kind": "oracle",
            "sample": f"full SMP-PCA pipeline on the first {d_s} of {c['d']} rows "
                      f"({gbytes:.2f} GB of FP32 input), {dt:.1f} s"}


def cpu_baseline_sketch(A, B, c, seed, rows):
    """The oracle's single pass (Alg. 1 step 2: Pi drawn from the counter,
    FP64 products, exact column norms) over the first `rows` rows of A and B.
    At this size the oracle's downstream stages alone (a dense 4,096^2 SVD and
    the per-row solves) take over a minute of host time, so the bounded sample
    is the pass, which is also what the metric's GB/s measures."""
    from oracle import sketch as osk

    d_s = min(rows, c["d"])
    a = A[:d_s].cpu().numpy()
    b = B[:d_s].cpu().numpy()
    t0 = time.perf_counter()
    osk.sketch(a, b, seed, c["k"])
    dt = time.perf_counter() - t0
    gbytes = 4.0 * d_s * (c["n1"] + c["n2"]) / 1e9
    return {"value": gbytes / dt, "unit": "GB/s", "cores": _threads(), "kind": "oracle",
            "sample": f"oracle sketch pass (Pi generation, FP64 products, column norms) over the first {d_s} of "
                      f"{c['d']} rows ({gbytes:.2f} GB of FP32 input), {dt:.1f} s; the oracle's downstream stages "
                      f"are not in the sample"}


def product_fp64(A, B, chunk=1 << 16):
    """A^T B in FP64 on the device, accumulated over row chunks (B None: A^T A)."""
    import torch
    M = torch.zeros(A.shape[1], (A if B is None else B).shape[1], dtype=torch.float64, device=A.device)
    for l0 in range(0, A.shape[0], chunk):
        a = A[l0:l0 + chunk].double()
        M += a.T @ (a if B is None else B[l0:l0 + chunk].double())
    return M


def spectral_error(M, U, s, V, iters=60):
    """||M - U diag(s) V^T||_2 / ||M||_2 by power iteration in FP64 on the
    device (evaluation only, outside the timed region)."""
    import torch
    E = M - (U * s[None, :]) @ V.T

    def norm2(X):
        g = torch.Generator(device=X.device).manual_seed(7)
        v = torch.randn(X.shape[1], dtype=torch.float64, device=X.device, generator=g)
        for _ in range(iters):
            v = X.T @ (X @ v)
            v /= torch.linalg.vector_norm(v)
        return torch.linalg.vector_norm(X @ v).item()

    return norm2(E) / norm2(M)


def run_leg(ctx, api, A, B, c, seed, prec, steps, warmup, same=False, sketch="gaussian"):
    import torch
    dev = A.device
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], seed=seed, prec=prec, b_is_a=same,
                        sketch=sketch)
    U = torch.empty(c["n1"], c["r"], dtype=torch.float64, device=dev)
    V = torch.empty(c["n2"], c["r"], dtype=torch.float64, device=dev)
    s = torch.empty(c["r"], dtype=torch.float64, device=dev)
    Bx = A if same else B
    # inside the timed region only the sketch pass is bracketed by HIP events
    # (the roofline's kernel time); each event pair leaves the GPU idle for
    # about 10 us at a stage boundary, so the other stages are timed after it
    ctx.smp_set_timing(2)
    for _ in range(warmup):
        ctx.smp_solve(p, A, Bx, U, V, s)
    torch.cuda.synchronize()
    lat, sketch = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        ctx.smp_solve(p, A, Bx, U, V, s)          # synchronises at its end
        lat.append((time.perf_counter() - ts) * 1e3)
        sketch.append(ctx.smp_stage_times()["sketch"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / steps * 1e3
    in_bytes = 4.0 * c["d"] * (c["n1"] + (0 if same else c["n2"]))
    flops = (2.0 * c["k"] + 4.0) * c["d"] * (c["n1"] + (0 if same else c["n2"]))
    # stage breakdown: further solves with every stage bracketed (not timed)
    ctx.smp_set_timing(1)
    stages = []
    for _ in range(max(1, min(steps, 5))):
        ctx.smp_solve(p, A, Bx, U, V, s)
        stages.append(ctx.smp_stage_times())
    ctx.smp_set_timing(0)
    avg = {k: sum(st[k] for st in stages) / len(stages) for k in stages[0]}
    avg["sketch"] = sum(sketch) / len(sketch)
    return dict(p=p, ms_step=ms_step, in_bytes=in_bytes, flops=flops, avg=avg, lat=lat, out=(U, s, V))


def leg_summary(leg, err=None):
    sk = leg["avg"]["sketch"]
    out = {"ms_per_step": round(leg["ms_step"], 4), "solves_per_s": round(1e3 / leg["ms_step"], 3),
           "input_gbps": round(leg["in_bytes"] / (leg["ms_step"] / 1e3) / 1e9, 2),
           "latency_ms": {"p50": round(pct(leg["lat"], 50), 4), "p99": round(pct(leg["lat"], 99), 4)},
           "stages_ms": {k: round(v, 4) for k, v in leg["avg"].items()},
           "sketch_pass_gbps": round(leg["in_bytes"] / (sk / 1e3) / 1e9, 2),
           "sketch_pass_hbm_frac": round(leg["in_bytes"] / (sk / 1e3) / 1e9 / PEAK_HBM_GBPS, 4),
           "sketch_pass_tflops": round(leg["flops"] / (sk / 1e3) / 1e12, 2)}
    if err is not None:
        out["spectral_error"] = err
    return out


def roofline(leg, prec, traffic_name, kernel):
    """The sketch pass against the roofline that bounds it at this size:
    the matrix cores when flops / peak exceeds bytes / HBM peak, else HBM."""
    sk = leg["avg"]["sketch"] / 1e3
    peak_mfma = {"bf16": PEAK_BF16_MFMA_TFLOPS, "fp8": PEAK_FP8_MFMA_TFLOPS, "fp32": PEAK_FP32_MFMA_TFLOPS}[prec]
    tflops = leg["flops"] / sk / 1e12
    gbps = leg["in_bytes"] / sk / 1e9
    mfma_bound = leg["flops"] / (peak_mfma * 1e12) > leg["in_bytes"] / (PEAK_HBM_GBPS * 1e9)
    base = {"traffic": recorded_traffic(traffic_name), "kernel": kernel, "kernel_ms": round(sk * 1e3, 4),
            "bytes_per_launch": leg["in_bytes"], "flops_per_launch": leg["flops"],
            "hbm_gbps": round(gbps, 2), "hbm_frac": round(gbps / PEAK_HBM_GBPS, 4),
            "mfma_tflops": round(tflops, 2), "mfma_frac": round(tflops / peak_mfma, 4)}
    if mfma_bound:
        return dict({"bound": "mfma", "achieved": round(tflops, 2), "peak": peak_mfma, "unit": "TFLOP/s",
                     "frac": round(tflops / peak_mfma, 4)}, **base)
    return dict({"bound": "hbm", "achieved": round(gbps, 2), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                 "frac": round(gbps / PEAK_HBM_GBPS, 4)}, **base)


KERNELS = {
    "bf16": "BF16 sketch pass: per Pi window pi_store_bf16_kernel then sketch_bf16_stored_kernel "
            "(v_mfma_f32_16x16x32_bf16), then the tail launch, timed together",
    "fp8": "FP8 sketch pass, fragment form at k > 416: per window pi_store_fp8_kernel, quantize_fp8_kernel "
           "(the data once into E4M3 operand fragments with E8M0 scales and norms), fp8_norm_reduce_kernel and "
           "sketch_fp8_frag_kernel (v_mfma_scale_f32_16x16x128_f8f6f4), timed together; at k <= 416 the stored-Pi "
           "form (pi_store_fp8_kernel, sketch_fp8_stored_kernel, tail launch)",
    "fp32": "sketch_kernel (v_mfma_f32_16x16x4f32, Pi regenerated per tile)",
}


def _pools(spec, count, d, n, seed, dev):
    import smp_inputs
    return [smp_inputs.latent_pair(d, n, n, spec["R"], spec["sigma"], spec["alpha"], seed + 7919 * i, device=dev)
            for i in range(count)]


def run_mix(api, jobs, pools, large_pool, prec, workers, arrivals=None, budget=0):
    """Run the jobs through one server (admission within `budget` bytes, 0:
    none); arrivals (seconds from start) or all at once. Returns timing and
    latency figures."""
    import threading

    import torch
    dev = pools[0][0].device
    work = []
    for j in jobs:
        A, B = large_pool if j["large"] else pools[j["pool"]]
        d, n, r = j["d"], j["n"], j["r"]
        p = api.make_params(d, n, n, j["k"], r, T=10, seed=j["seed"], prec=prec)
        outs = (torch.empty(n, r, dtype=torch.float64, device=dev), torch.empty(n, r, dtype=torch.float64, device=dev),
                torch.empty(r, dtype=torch.float64, device=dev))
        work.append((p, A[:d, :n], B[:d, :n], outs, 8.0 * d * n, j["large"]))
    torch.cuda.synchronize()
    srv = api.Server(0, workers=workers, hbm_budget=int(budget))
    ids = [None] * len(work)
    results = [None] * len(work)

    def waiter():
        for i in range(len(work)):
            while ids[i] is None:
                time.sleep(0.0002)
            results[i] = srv.wait(ids[i])

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    for i, (p, A, B, outs, _, _) in enumerate(work):
        if arrivals is not None:
            delay = t0 + arrivals[i] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
        ids[i] = srv.submit(p, A, B, *outs)
    th.join()
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat = [r["queue_ms"] + r["run_ms"] for r in results]
    out = {"jobs": len(work), "failed": sum(r["status"] != 0 for r in results), "wall_s": round(wall, 4),
           "solves_per_s": round(len(work) / wall, 2),
           "input_gbps": round(sum(w[4] for w in work) / wall / 1e9, 2),
           "latency_ms": {"p50": round(pct(lat, 50), 3), "p99": round(pct(lat, 99), 3)},
           "run_ms": {"p50": round(pct([r["run_ms"] for r in results], 50), 3),
                      "p99": round(pct([r["run_ms"] for r in results], 99), 3)},
           "max_running": st["max_running"]}
    if budget:
        out["hbm_budget_gb"] = round(budget / 1e9, 1)
        out["max_in_use_gb"] = round(st["max_budget_in_use"] / 1e9, 2)
    big = [l for l, w in zip(lat, work) if w[5]]
    if big:
        small = [l for l, w in zip(lat, work) if not w[5]]
        out["latency_ms_large"] = {"p50": round(pct(big, 50), 3), "p99": round(pct(big, 99), 3), "count": len(big)}
        out["latency_ms_small"] = {"p50": round(pct(small, 50), 3), "p99": round(pct(small, 99), 3)}
    return out


def run_batch_group(api, jobs, pools, prec, workers, graph=True):
    """The jobs through smp_solve_batch_group: steps 2-4 on worker threads,
    then WAltMin for all jobs grouped."""
    import torch
    dev = pools[0][0].device
    work, batch = [], []
    for j in jobs:
        A, B = pools[j["pool"]]
        d, n, r = j["d"], j["n"], j["r"]
        p = api.make_params(d, n, n, j["k"], r, T=10, seed=j["seed"], prec=prec)
        outs = (torch.empty(n, r, dtype=torch.float64, device=dev), torch.empty(n, r, dtype=torch.float64, device=dev),
                torch.empty(r, dtype=torch.float64, device=dev))
        batch.append(dict(p=p, A=A[:d, :n], B=B[:d, :n], U=outs[0], V=outs[1], sigma=outs[2]))
        work.append(8.0 * d * n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, res = api.solve_batch_group(batch, workers=workers, graph=graph)
    wall = time.perf_counter() - t0
    return {"jobs": len(jobs), "failed": sum(r["status"] != 0 for r in res), "wall_s": round(wall, 4),
            "solves_per_s": round(len(jobs) / wall, 2), "input_gbps": round(sum(work) / wall / 1e9, 2),
            "graph": bool(graph)}


def run_sketch_group(api, jobs, pools):
    """The BF16 sketches alone of the batching mix's jobs: one smp_sketch per
    job on one context (the stored-Pi pass) against smp_sketch_group over all
    of them (the regenerating pass, jobs with the same kernel in one launch).
    Median of three timed runs after one warm-up each."""
    import torch
    dev = pools[0][0].device
    ctx = api.Context(0)
    P, As, Bs, outs, byts = [], [], [], [], 0.0
    for j in jobs:
        A, B = pools[j["pool"]]
        d, n, k = j["d"], j["n"], j["k"]
        P.append(api.make_params(d, n, n, k, j["r"], seed=j["seed"], prec=api.SMP_PREC_BF16))
        As.append(A[:d, :n])
        Bs.append(B[:d, :n])
        outs.append((torch.empty(n, k, device=dev), torch.empty(n, k, device=dev), torch.empty(n, device=dev),
                     torch.empty(n, device=dev)))
        byts += 8.0 * d * n

    def each():
        for p, A, B, o in zip(P, As, Bs, outs):
            ctx.smp_sketch(p, A, B, *o)

    def group():
        ctx.smp_sketch_group(P, As, Bs, *[[o[i] for o in outs] for i in range(4)])

    res = {}
    for name, f in (("per_job_ms", each), ("grouped_ms", group)):
        f()
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        res[name] = round(sorted(ts)[1] * 1e3, 2)
    del outs
    torch.cuda.empty_cache()
    res["per_job_gbps"] = round(byts / res["per_job_ms"] / 1e6, 1)
    res["grouped_gbps"] = round(byts / res["grouped_ms"] / 1e6, 1)
    res["what"] = ("the BF16 sketches alone of the batch jobs: one smp_sketch per job (stored-Pi pass) against one "
                   "smp_sketch_group call (regenerating pass, grouped launches)")
    return res


def mix_legs(api, args, pools, large_pool, dev):
    """The batching mix (512 jobs at once) and the serving mix (Poisson
    arrivals, 5% large jobs), each with BF16 and FP32 sketches."""
    import torch

    import smp_inputs
    b, sv = smp_inputs.BATCH, smp_inputs.SERVE
    seed = smp_inputs.SEED_BASE
    out = {}
    batch_jobs = smp_inputs.job_mix(b["jobs"], seed)
    g = torch.Generator().manual_seed(seed)
    arrivals, t = [], 0.0
    while True:
        t += float(torch.empty(1).exponential_(sv["rate_per_s"], generator=g))
        if t > args.serve_seconds:
            break
        arrivals.append(t)
    serve_jobs = smp_inputs.job_mix(len(arrivals), seed, large_frac=sv["large_frac"])
    for name, jobs, arr in (("batch", batch_jobs, None), ("serve", serve_jobs, arrivals)):
        if name == "serve" and large_pool is None:
            continue
        legs = {}
        budget = args.serve_budget_gb * 1e9 if name == "serve" else 0
        for leg, prec in (("bf16", api.SMP_PREC_BF16), ("fp32", api.SMP_PREC_FP32)):
            run_mix(api, jobs[:8], pools, large_pool, prec, args.workers)          # warm-up (workspaces, code)
            legs[leg] = run_mix(api, jobs, pools, large_pool, prec, args.workers, arr, budget)
        legs["bf16_vs_fp32_solves"] = round(legs["bf16"]["solves_per_s"] / legs["fp32"]["solves_per_s"], 3)
        if name == "batch":   # the same jobs with WAltMin grouped over all of them
            for leg, prec in (("bf16", api.SMP_PREC_BF16), ("fp32", api.SMP_PREC_FP32)):
                run_batch_group(api, jobs[:8], pools, prec, args.workers)          # warm-up
                legs["group_" + leg] = run_batch_group(api, jobs, pools, prec, args.workers)
            legs["sketch_group"] = run_sketch_group(api, jobs, pools)
        out[name] = legs
    out["batch"]["workload"] = (f"{b['jobs']} independent jobs submitted at once: d uniform in [10k, 200k], n1 = n2 "
                                f"uniform in [128, 2048], r in {{5, 10, 20}}, k = r * uniform{{4..20}}, T = 10, "
                                f"m = 4nr ln n; latent rank 10, noise 0.1, column scale (j+1)^-0.5; each job's own "
                                f"seed for Pi and the coins; inputs are top-left blocks of {b['pools']} resident "
                                f"200000 x 2048 pairs; {args.workers} server workers (bf16, fp32) or {args.workers} "
                                f"workers for steps 2-4 and WAltMin grouped over all jobs in one HIP graph per "
                                f"group of equal launch sequences (group_bf16, group_fp32)")
    if "serve" in out:
        out["serve"]["workload"] = (f"Poisson arrivals at {sv['rate_per_s']:.0f} jobs/s for {args.serve_seconds:.1f} s "
                                    f"({len(arrivals)} jobs): the batching mix plus {100 * sv['large_frac']:.0f}% large "
                                    f"jobs (d = 1M, n1 = n2 = 4096, r = 20, k = r * uniform{{4..20}}; the large "
                                    f"workload's matrices); {args.workers} server workers, admission within an HBM "
                                    f"budget of {args.serve_budget_gb:.0f} GB (each running job's workspace, inputs "
                                    f"and outputs)")
    return out


def main_mix(args):
    import torch

    import smp_inputs
    from paper_1610_06656_amd import api

    dev = torch.device("cuda:0")
    b, sv = smp_inputs.BATCH, smp_inputs.SERVE
    seed = smp_inputs.SEED_BASE
    pools = _pools(b, b["pools"], b["d"][1], b["n"][1], seed, dev)
    large_pool = None
    if args.workload == "serve":
        L = sv["large"]
        large_pool = _pools(sv, 1, L["d"], L["n"], seed, dev)[0]
    torch.cuda.synchronize()
    mix = mix_legs(api, args, pools, large_pool, dev)
    leg = mix[args.workload]
    out = {"metric": METRIC, "workload": args.workload, "value": leg["bf16"]["solves_per_s"], "unit": "solves/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": leg["workload"], "workers": args.workers}, "bf16": leg["bf16"], "fp32": leg["fp32"],
           "bf16_vs_fp32_solves": leg["bf16_vs_fp32_solves"]}
    out.update({k: v for k, v in leg.items() if k.startswith("group_")})
    print(json.dumps(out), flush=True)


def c2_legs(api, ctx, args, dev, seed, precs=("bf16", "fp32", "fp8")):
    """The d = 200,000, n = 2,000, k = 400 workload: its legs and errors."""
    import torch

    import smp_inputs
    c = C2
    A, B = smp_inputs.latent_pair(c["d"], c["n1"], c["n2"], c["R"], c["sigma"], c["alpha"], seed, device=dev)
    torch.cuda.synchronize()
    M = None if args.no_errors else product_fp64(A, B)
    prec_of = {"bf16": api.SMP_PREC_BF16, "fp32": api.SMP_PREC_FP32, "fp8": api.SMP_PREC_FP8}
    legs = {}
    for name in precs:
        leg = run_leg(ctx, api, A, B, c, seed, prec_of[name], args.steps, args.warmup)
        err = None if M is None else spectral_error(M, *leg["out"])
        legs[name] = dict(leg_summary(leg, err),
                          roofline=roofline(leg, name, f"sketch_{name}_c2_traffic", KERNELS[name]))
    return A, B, legs


def methods_c2(api, ctx, A, B, dev, seed, reps=5):
    """The paper's comparison (Section 4) at d = 200,000, n = 2,000, k = 400,
    r = 10 on the same matrices: the best rank-r error, LELA (two passes,
    exact entries), SVD(A~^T B~) and SMP-PCA (BF16 sketch); ms per solve and
    spectral error of each."""
    import torch
    c = C2
    M = product_fp64(A, B)
    sv = torch.linalg.svdvals(M)
    out = {"optimal_error": (sv[c["r"]] / sv[0]).item()}
    for name, fn, prec in (("smp_pca_bf16", ctx.smp_solve, api.SMP_PREC_BF16), ("lela", ctx.smp_lela, api.SMP_PREC_FP32),
                           ("svd_sketch_bf16", ctx.smp_solve_svd_sketch, api.SMP_PREC_BF16)):
        p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], seed=seed, prec=prec)
        U = torch.empty(c["n1"], c["r"], dtype=torch.float64, device=dev)
        V = torch.empty(c["n2"], c["r"], dtype=torch.float64, device=dev)
        s = torch.empty(c["r"], dtype=torch.float64, device=dev)
        fn(p, A, B, U, V, s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn(p, A, B, U, V, s)
        torch.cuda.synchronize()
        out[name] = {"ms": round((time.perf_counter() - t0) / reps * 1e3, 3),
                     "error": float(torch.linalg.matrix_norm(M - (U * s[None, :]) @ V.T, 2) / sv[0])}
    return out


def sampler_legs(api, ctx, dev, reps=5):
    """smp_sample with one coin per grid entry (Alg. 1 step 3) against the
    row-wise multinomial draws of Appendix D, on squared norms with
    power-law column profiles, n1 = n2 = n, m = 4 n r ln n."""
    import numpy as np
    import torch
    from paper_1610_06656_amd.api import Omega
    out = []
    for n, r in ((2000, 10), (30000, 5), (100000, 5)):
        rng = np.random.default_rng(0)
        na2 = torch.from_numpy((rng.standard_normal(n) ** 2 * np.arange(1, n + 1) ** -0.8).astype(np.float32)).to(dev)
        nb2 = torch.from_numpy((rng.standard_normal(n) ** 2 * np.arange(1, n + 1) ** -0.5).astype(np.float32)).to(dev)
        row = {"n1": n, "n2": n, "r": r}
        for sampler in ("binomial", "multinomial"):
            if sampler == "binomial" and n > 30000:
                continue                      # 10^10 coins
            p = api.make_params(100, n, n, 8, r, sampler=sampler)
            om = Omega(n, n, int(p.m + n + 64 + 6 * p.m ** 0.5), dev)
            ctx.smp_sample(p, na2, nb2, om)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                nnz = ctx.smp_sample(p, na2, nb2, om)
            row[sampler + "_ms"] = round((time.perf_counter() - t0) / reps * 1e3, 3)
            row[sampler + "_omega"] = int(nnz)
            row["m"] = round(p.m, 1)
            del om
        out.append(row)
    return out


# Entry-wise sketch (matrices given as entries in any order): the accumulation
# kernel regenerates Pi per entry, so it is bound by the vector ALUs. Its peak
# in entry-rows (one entry times one sketch row) per second comes from the
# published FP32 vector rate, 157.3 TFLOP/s = 78.65 T lane-operations per
# second (an FMA counted once; 128 per clock per CU at 2.4 GHz on 256 CUs):
# one Philox4x32-10 call with its Box-Muller transform and the four
# multiply-adds takes 70 of them per lane (10 rounds of two 32x32->64-bit
# products and two three-input XORs, 26 for the two Box-Muller pairs, 4 FMAs)
# and serves 4 sketch rows; the SRHT takes 4 per entry-row (AND, popcount,
# sign select, add). Transcendentals and 64-bit products issue slower than
# that rate, so this peak is an upper bound for the instruction mix.
VALU_LANE_OPS_PER_S = 157.3e12 / 2
SPARSE_PEAK_ENTRY_ROWS = {"gauss_fp32": VALU_LANE_OPS_PER_S * 4 / 70, "gauss_bf16": VALU_LANE_OPS_PER_S * 4 / 70,
                          "srht": VALU_LANE_OPS_PER_S / 4}


def sparse_legs(api, ctx, dev, seed, reps=5, errors=True):
    """Entry pushes (smp_sketch_push_coo, entries in a random arrival order) of
    the URL-reputation shape (Table 1: d = 792,145, two sets of 10,000
    features, k = 2,000; ~20 M entries each) and the NIPS-BW shape (12,419
    words x 750 + 750 papers, k = 400), then smp_solve_sketched, for the
    Gaussian sketch in FP32 and BF16 and the SRHT; spectral errors against
    A^T B formed by scipy.sparse on the host (outside the timed region)."""
    import numpy as np
    import scipy.sparse
    import torch

    from smp_inputs import sparse as spin
    out = {}
    for cname in ("s3_url", "s2_bow"):
        c = spin.SPARSE_CONFIGS[cname]
        A, B = spin.sparse_pair(c, seed)
        d, n1, n2, k, r = c["d"], c["n1"], c["n2"], c["k"], c["r"]
        dA = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in A]
        dB = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in B]
        nnz = len(A[0]) + len(B[0])
        M = None
        if errors:
            SA = scipy.sparse.csr_matrix((A[2].astype(np.float64), (A[0], A[1])), shape=(d, n1))
            SB = scipy.sparse.csr_matrix((B[2].astype(np.float64), (B[0], B[1])), shape=(d, n2))
            M = torch.from_numpy((SA.T @ SB).toarray()).to(dev)
            del SA, SB
        row = {"workload": ("URL-reputation shape" if cname == "s3_url" else "NIPS-BW shape")
               + f": d={d}, n1={n1}, n2={n2}, k={k}, r={r}, T={c['T']}, topic-model counts, entries in random order",
               "nnz_a": len(A[0]), "nnz_b": len(B[0])}
        At = torch.empty(n1, k, device=dev)
        Bt = torch.empty(n2, k, device=dev)
        na = torch.empty(n1, device=dev)
        nb = torch.empty(n2, device=dev)
        U = torch.empty(n1, r, dtype=torch.float64, device=dev)
        V = torch.empty(n2, r, dtype=torch.float64, device=dev)
        s = torch.empty(r, dtype=torch.float64, device=dev)
        for name, kw in (("gauss_fp32", {}), ("gauss_bf16", {"prec": api.SMP_PREC_BF16}), ("srht", {"sketch": "srht"})):
            p = api.make_params(d, n1, n2, k, r, T=c["T"], seed=seed, **kw)

            def push_all():
                st = ctx.smp_sketch_begin(p)
                acc = 0.0
                try:
                    ctx.smp_sketch_push_coo(st, api.SMP_MAT_A, *dA)
                    acc += ctx.smp_stage_times()["sketch"]
                    ctx.smp_sketch_push_coo(st, api.SMP_MAT_B, *dB)
                    acc += ctx.smp_stage_times()["sketch"]
                    ctx.smp_sketch_end(st, At, Bt, na, nb)
                    torch.cuda.synchronize()
                finally:
                    ctx.smp_sketch_free(st)
                return acc

            ctx.smp_set_timing(2)
            push_all()
            walls, kern = [], []
            for _ in range(reps):
                t0 = time.perf_counter()
                kern.append(push_all())
                walls.append(time.perf_counter() - t0)
            ctx.smp_set_timing(0)
            wall, kt = pct(walls, 50), pct(kern, 50) / 1e3
            er = nnz * k / kt
            peak = SPARSE_PEAK_ENTRY_ROWS[name]
            leg = {"ms_per_sketch": round(wall * 1e3, 3), "accumulate_ms": round(kt * 1e3, 3),
                   "entries_per_s": round(nnz / wall, 1),
                   "roofline": {"bound": "alu", "achieved": round(er / 1e9, 2), "peak": round(peak / 1e9, 2),
                                "unit": "G entry-rows/s", "frac": round(er / peak, 4),
                                "kernel": "sp_sketch_kernel + sp_long_reduce_kernel of both pushes "
                                          "(after the radix sort)", "kernel_ms": round(kt * 1e3, 3)}}
            ctx.smp_solve_sketched(p, At, Bt, na, nb, U, V, s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.smp_solve_sketched(p, At, Bt, na, nb, U, V, s)
            leg["solve_sketched_ms"] = round((time.perf_counter() - t0) / reps * 1e3, 3)
            if M is not None:
                leg["spectral_error"] = spectral_error(M, U, s, V)
            row[name] = leg
        if M is not None and cname == "s2_bow":
            sv = torch.linalg.svdvals(M)
            row["optimal_error"] = float(sv[r] / sv[0])
        out[cname] = row
        del M, dA, dB, At, Bt
        torch.cuda.empty_cache()
    return out


def main_sparse(args):
    import torch

    import smp_inputs
    from paper_1610_06656_amd import api

    dev = torch.device("cuda:0")
    ctx = api.Context(0)
    sp = sparse_legs(api, ctx, dev, smp_inputs.SEED_BASE, reps=max(1, args.steps), errors=not args.no_errors)
    head = sp["s3_url"]["gauss_fp32"]
    out = {"metric": "entries/s of the entry-wise sketch (both matrices) + ALU roofline of its accumulation kernel",
           "value": head["entries_per_s"], "unit": "entries/s", "n_gpus": 1, "steps": max(1, args.steps),
           "warmup": 1, "ms_per_step": head["ms_per_sketch"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": sp["s3_url"]["workload"]}, "roofline": head["roofline"]}
    out.update(sp)
    print(json.dumps(out), flush=True)


def main_c2(args):
    import torch

    import smp_inputs
    from paper_1610_06656_amd import api

    dev = torch.device("cuda:0")
    seed = smp_inputs.SEED_BASE
    ctx = api.Context(0)
    precs = [x for x in args.legs.split(",") if x in ("bf16", "fp32", "fp8")]
    assert "bf16" in precs, "--legs must include bf16"
    A, B, legs = c2_legs(api, ctx, args, dev, seed, precs=precs)
    c = C2
    bf = legs["bf16"]
    out = {"metric": METRIC, "value": bf["input_gbps"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": bf["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "SMP-PCA end to end, d=200000, n1=n2=2000, k=400, r=10, T=10, m=4nr ln n",
                      "d": c["d"], "n1": c["n1"], "n2": c["n2"], "k": c["k"], "r": c["r"], "T": c["T"]},
           "roofline": bf["roofline"]}
    out.update(legs)
    if "fp32" in legs:
        out["bf16_vs_fp32_solves"] = round(legs["fp32"]["ms_per_step"] / bf["ms_per_step"], 3)
    if args.copy_calibration:
        copy_calibration(dev, out)
    if not args.no_cpu_baseline:
        p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], seed=seed)
        out["cpu_baseline"] = cpu_baseline_pipeline(A, B, c, p.m, seed, args.cpu_rows)
    print(json.dumps(out), flush=True)


def copy_calibration(dev, out):
    """One plain device copy of 2^30 bytes: the reference dispatch that scales
    rocprofv3's FETCH_SIZE / WRITE_SIZE readings to bytes."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_calibration_bytes"] = 1 << 30


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (sharding across GPUs "
                                   "is not built)"}))
        sys.exit(2)
    if args.workload in ("batch", "serve"):
        return main_mix(args)
    if args.workload == "sparse":
        return main_sparse(args)
    if args.workload == "c2":
        return main_c2(args)
    import torch

    import smp_inputs
    from paper_1610_06656_amd import api

    dev = torch.device("cuda:0")
    seed = smp_inputs.SEED_BASE
    legs_wanted = [x for x in args.legs.split(",") if x]
    assert legs_wanted and all(x in LEGS for x in legs_wanted), f"--legs: a subset of {LEGS}"
    head = "bf16" if "bf16" in legs_wanted else legs_wanted[0]   # profiling runs may time one other leg only
    c = C3
    A, B = smp_inputs.latent_pair(c["d"], c["n1"], c["n2"], c["R"], c["sigma"], c["alpha"], seed, device=dev)
    torch.cuda.synchronize()
    ctx = api.Context(0)
    prec_of = {"bf16": api.SMP_PREC_BF16, "fp8": api.SMP_PREC_FP8, "fp32": api.SMP_PREC_FP32, "ab": api.SMP_PREC_BF16,
               "srht": api.SMP_PREC_FP32}
    tune = {}
    if args.tune:   # launch shapes measured by smp_tune_sketch before any timed region; the legs then use them
        for name in legs_wanted:
            if name in ("bf16", "fp8", "ab"):
                p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], seed=seed,
                                    prec=prec_of[name], b_is_a=(name == "ab"))
                t0 = time.perf_counter()
                cap, spl, ms = ctx.smp_tune_sketch(p, A, None if name == "ab" else B)
                tune[name] = {"cap": cap, "splits": spl, "ms_per_launch": round(ms, 4),
                              "tuning_s": round(time.perf_counter() - t0, 3)}
    runs = {}
    for name in legs_wanted:
        runs[name] = run_leg(ctx, api, A, B, c, seed, prec_of[name], args.steps, args.warmup, same=(name == "ab"),
                             sketch="srht" if name == "srht" else "gaussian")
    # spectral errors (outside every timed region)
    errs = {}
    if not args.no_errors:
        M = product_fp64(A, B)
        for name in legs_wanted:
            if name != "ab":
                errs[name] = spectral_error(M, *runs[name]["out"])
        del M
        if "ab" in runs:
            Maa = product_fp64(A, None)
            errs["ab"] = spectral_error(Maa, *runs["ab"]["out"])
            del Maa
        torch.cuda.empty_cache()
    legs = {}
    for name in legs_wanted:
        if name == "srht":       # additions on the vector ALUs, no matrix-core work
            legs[name] = dict(leg_summary(runs[name], errs.get(name)),
                              kernel="srht_kernel: length-512 fast Walsh-Hadamard transforms of row chunks (FP32)")
            continue
        prec = "bf16" if name == "ab" else name
        legs[name] = dict(leg_summary(runs[name], errs.get(name)),
                          roofline=roofline(runs[name], prec, f"sketch_{name}_c3_traffic", KERNELS[prec]))
    bf = runs[head]
    value = bf["in_bytes"] / (bf["ms_step"] / 1e3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "value_is": "input bytes 4 d (n1+n2) per second of the whole BF16 smp_solve (inputs resident in HBM); "
                    "the sketch pass alone: roofline.hbm_gbps and roofline.mfma_tflops",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(bf["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "SMP-PCA end to end, dense latent-rank-20 A and B (noise 0.05, column scale "
                               "(j+1)^-0.7), d=1000000, n1=n2=4096, k=1024, r=20, T=10, m=4nr ln n; BF16 sketch "
                               "GEMM (FP32 accumulate, FP32 compensated norms), FP64 sampling weights, estimates "
                               "and WAltMin", "d": c["d"], "n1": c["n1"], "n2": c["n2"], "k": c["k"],
                   "r": c["r"], "T": c["T"], "m": round(bf["p"].m, 3), "input_gb": round(bf["in_bytes"] / 1e9, 3)},
        "roofline": legs[head]["roofline"],
        "solves_per_s": round(1e3 / bf["ms_step"], 3),
        "latency_ms": legs[head]["latency_ms"],
        "spectral_error": errs.get(head),
    }
    out.update(legs)
    if tune:
        out["tune"] = tune
    if "fp32" in runs and head == "bf16":
        out["bf16_vs_fp32_solves"] = round(runs["fp32"]["ms_step"] / bf["ms_step"], 3)
    if args.copy_calibration:
        copy_calibration(dev, out)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_sketch(A, B, c, seed, args.cpu_rows or 200_000)
    if not args.no_c2:
        A2, B2, c2 = c2_legs(api, ctx, args, dev, seed, precs=("bf16", "fp32"))
        c2["bf16_vs_fp32_solves"] = round(c2["fp32"]["ms_per_step"] / c2["bf16"]["ms_per_step"], 3)
        c2["workload"] = "d=200000, n1=n2=2000, k=400, r=10, T=10; latent rank 10, noise 0.1, column scale (j+1)^-0.5"
        if not args.no_errors:
            c2["methods"] = methods_c2(api, ctx, A2, B2, dev, seed)
        out["c2"] = c2
        del A2, B2
        out["sampler"] = sampler_legs(api, ctx, dev)
    if not args.no_sparse:
        out["sparse"] = sparse_legs(api, ctx, dev, seed, errors=not args.no_errors)
    if not args.no_mix:
        import smp_inputs as si
        b = si.BATCH
        torch.cuda.empty_cache()
        pools = _pools(b, b["pools"], b["d"][1], b["n"][1], seed, dev)
        torch.cuda.synchronize()
        out.update(mix_legs(api, args, pools, (A, B), dev))
        del pools
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

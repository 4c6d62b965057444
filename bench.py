"""Benchmark of the SMP-PCA hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one smp_solve (Alg. 1 end to end: sketch pass, sampling, rescaled-JL
estimates, WAltMin, canonical form) over the dense FP32 workload
d = 200,000, n1 = n2 = 2,000, k = 400, r = 10, T = 10, m = 4 n r ln n
(latent rank 10, noise 0.1, column scaling (j+1)^-0.5), with A and B already
resident in HBM. `value` is input bytes consumed per second, 4 d (n1+n2) / t,
of the BF16-sketch solve (sketch GEMM operands rounded to bfloat16, FP32
accumulation, FP64 WAltMin); the same solve with the FP32 sketch ("fp32") and
with the FP8 E4M3 block-scaled sketch ("fp8") is timed beside it, and each
leg's spectral error is reported.

Also reported: the dominant kernel's roofline (the sketch pass, timed with HIP
events on the library's stream), per-stage times, solves/s with p50/p99
latency, and the FP64 CPU oracle timed on the host.
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
CFG = dict(d=200_000, n1=2000, n2=2000, R=10, sigma=0.1, alpha=0.5, k=400, r=10, T=10)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="rows of the CPU-oracle sample (0: all d rows)")
    ap.add_argument("--workload", choices=("c2", "batch", "serve"), default="c2",
                    help="c2: the headline solve (default); batch: 512 jobs of the batching mix through the "
                         "server; serve: Poisson arrivals of the serving mix")
    ap.add_argument("--workers", type=int, default=4, help="server worker threads (batch, serve)")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="arrival window of the serve workload")
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


def cpu_baseline(A, B, c, m, seed, rows):
    """The oracle as it stands (FP64 numpy) on a bounded sample of the same
    workload: the first `rows` rows of A and B, the full downstream pipeline."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import solve as osolve

    d_s = min(rows or c["d"], c["d"])
    a = A[:d_s].cpu().numpy()
    b = B[:d_s].cpu().numpy()
    t0 = time.perf_counter()
    osolve.smp_pca(a, b, c["r"], c["k"], m, c["T"], seed)
    dt = time.perf_counter() - t0
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    gbytes = 4.0 * d_s * (c["n1"] + c["n2"]) / 1e9
    return {"value": gbytes / dt, "unit": "GB/s", "cores": int(threads), "kind": "oracle",
            "sample": f"full SMP-PCA pipeline on the first {d_s} of {c['d']} rows "
                      f"({gbytes:.2f} GB of FP32 input), {dt:.1f} s"}


def spectral_error(A, B, U, s, V, iters=60):
    """||A^T B - U diag(s) V^T||_2 / ||A^T B||_2 by power iteration in FP64
    on the device (evaluation only, outside the timed region)."""
    import torch
    M = A.double().T @ B.double()
    E = M - (U * s[None, :]) @ V.T

    def norm2(X):
        g = torch.Generator(device=X.device).manual_seed(7)
        v = torch.randn(X.shape[1], dtype=torch.float64, device=X.device, generator=g)
        for _ in range(iters):
            v = X.T @ (X @ v)
            v /= torch.linalg.vector_norm(v)
        return torch.linalg.vector_norm(X @ v).item()

    return norm2(E) / norm2(M)


def run_leg(ctx, api, A, B, c, seed, prec, steps, warmup):
    import torch
    dev = A.device
    p = api.make_params(c["d"], c["n1"], c["n2"], c["k"], c["r"], T=c["T"], seed=seed, prec=prec)
    U = torch.empty(c["n1"], c["r"], dtype=torch.float64, device=dev)
    V = torch.empty(c["n2"], c["r"], dtype=torch.float64, device=dev)
    s = torch.empty(c["r"], dtype=torch.float64, device=dev)
    # inside the timed region only the sketch pass is bracketed by HIP events
    # (the roofline's kernel time); each event pair leaves the GPU idle for
    # about 10 us at a stage boundary, so the other stages are timed after it
    ctx.smp_set_timing(2)
    for _ in range(warmup):
        ctx.smp_solve(p, A, B, U, V, s)
    torch.cuda.synchronize()
    lat, sketch = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        ctx.smp_solve(p, A, B, U, V, s)          # synchronises at its end
        lat.append((time.perf_counter() - ts) * 1e3)
        sketch.append(ctx.smp_stage_times()["sketch"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / steps * 1e3
    in_bytes = 4.0 * c["d"] * (c["n1"] + c["n2"])
    # stage breakdown: further solves with every stage bracketed (not timed)
    ctx.smp_set_timing(1)
    stages = []
    for _ in range(max(1, min(steps, 5))):
        ctx.smp_solve(p, A, B, U, V, s)
        stages.append(ctx.smp_stage_times())
    ctx.smp_set_timing(0)
    avg = {k: sum(st[k] for st in stages) / len(stages) for k in stages[0]}
    avg["sketch"] = sum(sketch) / len(sketch)
    return dict(p=p, ms_step=ms_step, in_bytes=in_bytes, avg=avg, lat=lat,
                err=spectral_error(A, B, U, s, V))


def leg_summary(leg):
    sk = leg["avg"]["sketch"]
    return {"ms_per_step": round(leg["ms_step"], 4), "solves_per_s": round(1e3 / leg["ms_step"], 3),
            "latency_ms": {"p50": round(pct(leg["lat"], 50), 4), "p99": round(pct(leg["lat"], 99), 4)},
            "stages_ms": {k: round(v, 4) for k, v in leg["avg"].items()},
            "sketch_pass_gbps": round(leg["in_bytes"] / (sk / 1e3) / 1e9, 2),
            "sketch_pass_hbm_frac": round(leg["in_bytes"] / (sk / 1e3) / 1e9 / PEAK_HBM_GBPS, 4),
            "spectral_error": leg["err"]}


def _pools(spec, count, d, n, seed, dev):
    import smp_inputs
    return [smp_inputs.latent_pair(d, n, n, spec["R"], spec["sigma"], spec["alpha"], seed + 7919 * i, device=dev)
            for i in range(count)]


def run_mix(api, jobs, pools, large_pool, prec, workers, arrivals=None):
    """Run the jobs through one server; arrivals (seconds from start) or all
    at once. Returns timing and latency figures."""
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
    srv = api.Server(0, workers=workers)
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
    big = [l for l, w in zip(lat, work) if w[5]]
    if big:
        small = [l for l, w in zip(lat, work) if not w[5]]
        out["latency_ms_large"] = {"p50": round(pct(big, 50), 3), "p99": round(pct(big, 99), 3), "count": len(big)}
        out["latency_ms_small"] = {"p50": round(pct(small, 50), 3), "p99": round(pct(small, 99), 3)}
    return out


def main_mix(args):
    import torch

    import smp_inputs
    from paper_1610_06656_amd import api

    dev = torch.device("cuda:0")
    b, sv = smp_inputs.BATCH, smp_inputs.SERVE
    seed = smp_inputs.SEED_BASE
    pools = _pools(b, b["pools"], b["d"][1], b["n"][1], seed, dev)
    if args.workload == "batch":
        jobs = smp_inputs.job_mix(b["jobs"], seed)
        large_pool, arrivals = None, None
        desc = (f"{b['jobs']} independent jobs: d uniform in [10k, 200k], n1 = n2 uniform in [128, 2048], "
                f"r in {{5, 10, 20}}, k = r * uniform{{4..20}}, T = 10, m = 4nr ln n; latent rank 10, noise 0.1, "
                f"column scale (j+1)^-0.5; inputs are top-left blocks of {b['pools']} resident 200000 x 2048 pairs")
    else:
        L = sv["large"]
        large_pool = _pools(sv, 1, L["d"], L["n"], seed + 1, dev)[0]
        g = torch.Generator().manual_seed(seed)
        arrivals, t = [], 0.0
        while True:
            t += float(torch.empty(1).exponential_(sv["rate_per_s"], generator=g))
            if t > args.serve_seconds:
                break
            arrivals.append(t)
        jobs = smp_inputs.job_mix(len(arrivals), seed, large_frac=sv["large_frac"])
        desc = (f"Poisson arrivals at {sv['rate_per_s']:.0f} jobs/s for {args.serve_seconds:.1f} s: the batching mix "
                f"plus {100 * sv['large_frac']:.0f}% large jobs (d = 1M, n1 = n2 = 4096, r = 20; latent rank 20, "
                f"noise 0.05, column scale (j+1)^-0.7); inputs are blocks of resident pairs")
    torch.cuda.synchronize()
    legs = {}
    for name, prec in (("bf16", api.SMP_PREC_BF16), ("fp32", api.SMP_PREC_FP32)):
        run_mix(api, jobs[:8], pools, large_pool, prec, args.workers)          # warm-up (workspaces, code)
        legs[name] = run_mix(api, jobs, pools, large_pool, prec, args.workers, arrivals)
    out = {"metric": METRIC, "workload": args.workload, "value": legs["bf16"]["solves_per_s"], "unit": "solves/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": desc, "workers": args.workers}, "bf16": legs["bf16"], "fp32": legs["fp32"]}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (sharding across GPUs "
                                   "is not built)"}))
        sys.exit(2)
    if args.workload != "c2":
        return main_mix(args)
    import torch

    import smp_inputs
    from paper_1610_06656_amd import api

    dev = torch.device("cuda:0")
    c = CFG
    seed = smp_inputs.SEED_BASE
    A, B = smp_inputs.latent_pair(c["d"], c["n1"], c["n2"], c["R"], c["sigma"], c["alpha"], seed, device=dev)
    torch.cuda.synchronize()
    ctx = api.Context(0)

    fp32 = run_leg(ctx, api, A, B, c, seed, api.SMP_PREC_FP32, args.steps, args.warmup)
    bf16 = run_leg(ctx, api, A, B, c, seed, api.SMP_PREC_BF16, args.steps, args.warmup)
    fp8 = run_leg(ctx, api, A, B, c, seed, api.SMP_PREC_FP8, args.steps, args.warmup)

    in_bytes = bf16["in_bytes"]
    ms_step = bf16["ms_step"]
    value = in_bytes / (ms_step / 1e3) / 1e9
    sk_bf16 = bf16["avg"]["sketch"]
    sk_fp32 = fp32["avg"]["sketch"]
    sk_fp8 = fp8["avg"]["sketch"]
    flops = (2.0 * c["k"] + 4.0) * c["d"] * (c["n1"] + c["n2"])
    fp32_tflops = flops / (sk_fp32 / 1e3) / 1e12
    hbm_gbps = in_bytes / (sk_bf16 / 1e3) / 1e9
    p = bf16["p"]
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "SMP-PCA end to end, dense latent-rank-10 A and B (noise 0.1, column scale "
                               "(j+1)^-0.5), d=200000, n1=n2=2000, k=400, r=10, T=10, m=4nr ln n; BF16 sketch "
                               "GEMM (FP32 accumulate, FP32 compensated norms), FP64 sampling weights, "
                               "estimates and WAltMin", "d": c["d"], "n1": c["n1"], "n2": c["n2"], "k": c["k"],
                   "r": c["r"], "T": c["T"], "m": round(p.m, 3), "input_gb": round(in_bytes / 1e9, 3)},
        "roofline": {"bound": "hbm", "achieved": round(hbm_gbps, 2), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(hbm_gbps / PEAK_HBM_GBPS, 4),
                     "traffic": recorded_traffic("sketch_bf16_c2_traffic"),
                     "kernel": "BF16 sketch pass: pi_store_bf16_kernel, then sketch_bf16_stored_kernel "
                               "(v_mfma_f32_16x16x32_bf16) main and tail launch, timed together",
                     "mfma_tflops": round(flops / (sk_bf16 / 1e3) / 1e12, 2),
                     "mfma_frac": round(flops / (sk_bf16 / 1e3) / 1e12 / PEAK_BF16_MFMA_TFLOPS, 4),
                     "kernel_ms": round(sk_bf16, 4), "bytes_per_launch": in_bytes},
        "solves_per_s": round(1e3 / ms_step, 3),
        "latency_ms": {"p50": round(pct(bf16["lat"], 50), 4), "p99": round(pct(bf16["lat"], 99), 4)},
        "spectral_error": bf16["err"],
        "bf16": leg_summary(bf16),
        "fp32": dict(leg_summary(fp32), roofline={
            "bound": "mfma", "achieved": round(fp32_tflops, 3), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": round(fp32_tflops / PEAK_FP32_MFMA_TFLOPS, 4),
            "traffic": recorded_traffic("sketch_fp32_c2_traffic"),
            "kernel": "sketch_kernel (v_mfma_f32_16x16x4f32)", "kernel_ms": round(sk_fp32, 4),
            "flops_per_launch": flops}),
        "fp8": dict(leg_summary(fp8), roofline={
            "bound": "hbm", "achieved": round(in_bytes / (sk_fp8 / 1e3) / 1e9, 2), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(in_bytes / (sk_fp8 / 1e3) / 1e9 / PEAK_HBM_GBPS, 4), "traffic": recorded_traffic("sketch_fp8_c2_traffic"),
            "kernel": "FP8 sketch pass: pi_store_fp8_kernel, then sketch_fp8_stored_kernel "
                      "(v_mfma_scale_f32_16x16x128_f8f6f4) main and tail launch, timed together",
            "kernel_ms": round(sk_fp8, 4), "bytes_per_launch": in_bytes,
            "mfma_tflops": round(flops / (sk_fp8 / 1e3) / 1e12, 2),
            "mfma_frac": round(flops / (sk_fp8 / 1e3) / 1e12 / PEAK_FP8_MFMA_TFLOPS, 4)}),
        "bf16_vs_fp32_solves": round(fp32["ms_step"] / bf16["ms_step"], 3),
    }
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 1 << 30
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, B, c, p.m, seed, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

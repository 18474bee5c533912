"""Benchmark: time-to-OLS-accuracy of SPCG vs full-data PCG on one MI355X.

A step is one whole solve (nested SRHT sketch, FP64 QR preconditioner,
Stage I sketched PCG stages, Stage II full-data PCG until the stopping
test) of a synthetic least-squares problem already resident in HBM.
Prints one JSON line (see the design doc for every field).

    python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--workload cfg1|cfg2|cfg2fp8]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E

WORKLOADS = {
    "cfg1": dict(cfg=1, storage="f32",
                 desc="X = G diag(s), G Gaussian, s log-spaced 1..1e4; N=1000000, d=500; sigma=1; "
                      "X stored FP32"),
    "cfg2": dict(cfg=2, storage="bf16",
                 desc="X = T C, T Student-t(3), C = Q1 diag(s) Q2^T with s log-spaced 1..1e5; "
                      "N=4000000, d=1000; sigma=0.5; X stored BF16"),
    "cfg2fp8": dict(cfg=2, storage="fp8",
                    desc="X = T C, T Student-t(3), C = Q1 diag(s) Q2^T with s log-spaced 1..1e5; "
                         "N=4000000, d=1000; sigma=0.5; X stored FP8 e4m3 with per-column scales"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pred_error_vs_ols(p, beta, chunk=1 << 18):
    """||X (beta - beta_ols)|| / ||X beta_ols|| without forming beta_ols.

    With g = X^T (Y - X beta) and G = X^T X, X^T X (beta_ols - beta) = g, so
    ||X (beta - beta_ols)||^2 = g^T G^-1 g.  G, g and ||X beta|| are
    accumulated in FP64 over row chunks (no library call sees more than
    2^31 elements), then one Cholesky solve of the d x d system."""
    import torch
    d = p.d
    G = torch.zeros(d, d, dtype=torch.float64, device=beta.device)
    g = torch.zeros(d, dtype=torch.float64, device=beta.device)
    fit2 = 0.0
    b = beta.reshape(d, 1)
    for i in range(0, p.N, chunk):
        xb = p.x_f64(slice(i, min(i + chunk, p.N)))
        G += xb.T @ xb
        f = (xb @ b)[:, 0]
        g += xb.T @ (p.Y[i:i + chunk, 0] - f)
        fit2 += float(f.dot(f))
        del xb, f
    L = torch.linalg.cholesky(G)
    z = torch.cholesky_solve(g.unsqueeze(1), L)[:, 0]
    return float(torch.sqrt(torch.clamp(g.dot(z), min=0.0)) / max(fit2, 1e-300) ** 0.5)


def cpu_baseline(X, Y, d, n_sample):
    """The FP64 NumPy oracle's SPCG on the first n_sample rows, scaled by N/n_sample."""
    import numpy as np

    from oracle.spcg import spcg
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    Xs = X[:n_sample].double().cpu().numpy()
    Ys = Y[:n_sample, 0].cpu().numpy()
    t0 = time.perf_counter()
    spcg(Xs, Ys, seed=1)
    t = time.perf_counter() - t0
    return t, threads


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg1", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 16)
    ap.add_argument("--skip-check", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU row-sharded design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2607_25272_amd as spcg
    import workloads

    wl = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    log(f"generating {args.workload}")
    p = workloads.make_config(wl["cfg"], device=dev, storage=wl["storage"])
    torch.cuda.synchronize()
    N, d = p.N, p.d
    ctx = spcg.Context(0)
    beta = torch.zeros(d, dtype=torch.float64, device=dev)

    def solve(method, **kw):
        return spcg.spcg_solve(ctx, p.X, p.Y, beta=beta, col_scale=p.col_scale, method=method,
                               seed=1, **kw)

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst

    results = {}
    for method in ("spcg", "pcg"):
        log(f"{method}: warmup {args.warmup}")
        for _ in range(args.warmup):
            solve(method)
        torch.cuda.synchronize()
        log(f"{method}: timing {args.steps} solves")
        t0 = time.perf_counter()
        prod_ms, prod_n, last = 0.0, 0, None
        for _ in range(args.steps):
            _, st = solve(method, time_products=True)
            prod_ms += st["product_ms_sum"]
            prod_n += st["product_launches"]
            last = st
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        _, ph = solve(method, time_phases=True)
        torch.cuda.synchronize()
        rel = None
        if not args.skip_check:
            rel = pred_error_vs_ols(p, beta)
            torch.cuda.empty_cache()
        results[method] = dict(s=dt, stats=last, phases=ph, prod_ms=prod_ms, prod_n=prod_n, rel=rel)
        log(f"{method}: {dt * 1e3:.3f} ms/solve, K={last['K']} T1={last['T_stage1']} "
            f"T2={last['T_stage2']} rel={rel} phases sketch={ph['t_sketch_ms']:.3f} "
            f"precond={ph['t_precond_ms']:.3f} stage1={ph['t_stage1_ms']:.3f} "
            f"stage2={ph['t_stage2_ms']:.3f} ms")

    sp, pc = results["spcg"], results["pcg"]
    # roofline of the full-data product (Stage II / full PCG dual pass): one
    # read of X plus the FP64 response vector per launch
    bytes_per_launch = float(N) * d * p.X.element_size() + float(N) * 8.0
    n_launch = sp["prod_n"] + pc["prod_n"]
    avg_ms = (sp["prod_ms"] + pc["prod_ms"]) / max(n_launch, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        n_s = min(args.cpu_sample, N // 2)
        log(f"cpu baseline: oracle SPCG on {n_s} rows")
        t_cpu, threads = cpu_baseline(p.x_f64(slice(0, n_s)), p.Y, d, n_s)
        cpu = {"value": t_cpu * N / n_s, "unit": "s", "cores": threads, "kind": "oracle",
               "sample": f"FP64 NumPy oracle SPCG on the first {n_s} rows (d={d}) of the same "
                         f"workload took {t_cpu:.2f} s; value scaled linearly by N/{n_s}"}

    dtype = {"f32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}[wl["storage"]]
    out = {
        "metric": "time-to-OLS-accuracy (s) and PCG-product HBM GB/s, SPCG vs full PCG, 1 GPU",
        "value": sp["s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sp["s"] * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": wl["desc"], "tol": 5e-7, "a_i": 3, "r": 6 * d, "m_1": 4 * d,
                   "K": sp["stats"]["K"], "T_stage1": sp["stats"]["T_stage1"],
                   "T_stage2": sp["stats"]["T_stage2"]},
        "full_pcg_s": pc["s"],
        "full_pcg_iters": pc["stats"]["T_stage2"],
        "speedup_vs_full_pcg": pc["s"] / sp["s"],
        "rel_pred_error_vs_ols": {"spcg": sp["rel"], "pcg": pc["rel"]},
        "phases_ms": {m: {k: round(results[m]["phases"][k], 4) for k in
                          ("t_sketch_ms", "t_precond_ms", "t_stage1_ms", "t_stage2_ms", "t_total_ms")}
                      for m in results},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBPS) if achieved else None, "traffic": None,
                     "kernel": "product_kernel (SG mode, full data)",
                     "bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms,
                     "launches": n_launch},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

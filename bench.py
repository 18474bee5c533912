"""Benchmark: time-to-OLS-accuracy of SPCG vs full PCG on one MI355X.

A step is one whole solve (nested SRHT sketch, FP64 QR preconditioner,
Stage I sketched PCG stages, Stage II full-data PCG until the stopping
test) of a synthetic least-squares problem already resident in HBM.
Prints one JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2]
                    [--workload cfg1|cfg2|cfg2fp8|cfg1cs|cfg2cs|batched|learned|paper|tuned]

cfg1 (default)  N=1e6, d=500, FP32 storage
cfg2 / cfg2fp8  N=4e6, d=1000, BF16 / FP8-e4m3 storage (precision form)
cfg1cs / cfg2cs the same problems solved by SPCG-CS (CountSketch sketches,
                Sec. 4.3); SPCG-SRHT and full PCG are timed beside it
batched         256 independent problems, N in [5e4, 5e5], d in [32, 512],
                1..16 right-hand sides, FP32 (batched / multi-RHS form)
learned         N=2e6, d=256, 1% of rows scaled by 100: plain vs learned schedule
paper           the Sec. 4 / Table 1 setting (d=64, sigma^2=1e-8, m_1=8d,
                m_K=N/2, FP64), N=2^17..2^22: iteration counts and GPU times
tuned           the Sec. 4.3 setting (N=2^22, d=64, kappa=1e8): paper schedule,
                tuned sizes, theory-driven a_i, CountSketch, full PCG
"""
import argparse
import json
import os
import statistics
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
    "cfg1cs": dict(cfg=1, storage="f32", sketch="cs", base="cfg1",
                   desc="X = G diag(s), G Gaussian, s log-spaced 1..1e4; N=1000000, d=500; sigma=1; "
                        "X stored FP32; SPCG-CS (nested CountSketch)"),
    "cfg2cs": dict(cfg=2, storage="bf16", sketch="cs", base="cfg2",
                   desc="X = T C, T Student-t(3), C = Q1 diag(s) Q2^T with s log-spaced 1..1e5; "
                        "N=4000000, d=1000; sigma=0.5; X stored BF16; SPCG-CS (nested CountSketch)"),
    "learned": dict(cfg=4, storage="f32",
                    desc="X = G diag(s), s log-spaced 1..1e4, a seeded 1% of rows scaled by 100; "
                         "N=2000000, d=256; sigma=1; X stored FP32; plain vs learned schedule"),
    "batched": dict(desc="256 problems: N ~ U[5e4, 5e5], d ~ U[32, 512], column scales 1..kappa with "
                         "kappa log-uniform in [1e2, 1e5], k ~ U{1..16} right-hand sides; sigma=1; FP32"),
    "paper": dict(desc="Sec. 4 setting: X = G D, d=64, kappa in {1e4, 1e8}, sigma^2=1e-8, m_1=8d, "
                       "m_K=N/2, r=6d, a_i=3, FP64, N=2^17..2^22"),
    "tuned": dict(desc="Sec. 4.3 setting: X = G D, N=2^22, d=64, kappa=1e8, sigma^2=1e-8, FP64; SPCG (m_1=8d "
                       "doubling to N/2, a_i=3), the tuned schedule (2^10..2^16 then 2^20, a_i=4), theory-driven "
                       "a_i (Theorems 3.3/3.4, omega=0.5), SPCG-CS, and full PCG"),
}
METRIC = "time-to-OLS-accuracy (s) and PCG-product HBM GB/s, SPCG vs full PCG, 1 GPU"
# HBM bytes per launch of the full-data SG product from rocprofv3 PMC runs
# (2.0 x FETCH_SIZE + WRITE_SIZE, calibrated on a 1 GiB copy; the summary and
# commands are in profiles/hbm_traffic_sg_product_and_transform.txt).  Valid
# for the product kernel as profiled; workloads not profiled report null.
SG_TRAFFIC_BYTES = {"cfg1": 2.0103e9, "cfg2": 8.0366e9}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pred_error_vs_ols(p, beta, chunk=1 << 18):
    """max over right-hand sides of ||X (beta - beta_ols)|| / ||X beta_ols||,
    without forming beta_ols.

    With g = X^T (Y - X beta) and G = X^T X, X^T X (beta_ols - beta) = g, so
    ||X (beta - beta_ols)||^2 = g^T G^-1 g.  G, g and ||X beta|| are
    accumulated in FP64 over row chunks (no library call sees more than
    2^31 elements), then one Cholesky solve of the d x d system."""
    import torch
    d, k = p.d, p.k
    G = torch.zeros(d, d, dtype=torch.float64, device=beta.device)
    g = torch.zeros(d, k, dtype=torch.float64, device=beta.device)
    fit2 = torch.zeros(k, dtype=torch.float64, device=beta.device)
    b = beta.reshape(d, k)
    for i in range(0, p.N, chunk):
        xb = p.x_f64(slice(i, min(i + chunk, p.N)))
        G += xb.T @ xb
        f = xb @ b
        g += xb.T @ (p.Y[i:i + chunk] - f)
        fit2 += (f * f).sum(0)
        del xb, f
    L = torch.linalg.cholesky(G)
    z = torch.cholesky_solve(g, L)
    err = torch.sqrt(torch.clamp((g * z).sum(0), min=0.0)) / torch.sqrt(torch.clamp(fit2, min=1e-300))
    return float(err.max())


def cpu_baseline(X, Y, n_sample):
    """The FP64 NumPy oracle's SPCG on the first n_sample rows."""
    from oracle.spcg import spcg
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    Xs = X.double().cpu().numpy()
    Ys = Y[:n_sample, 0].cpu().numpy()
    t0 = time.perf_counter()
    spcg(Xs, Ys, seed=1)
    return time.perf_counter() - t0, threads


def roofline(avg_ms, launches, bytes_per_launch, kernel):
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBPS) if achieved else None, "traffic": None,
            "kernel": kernel, "bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms,
            "launches": launches}


def timed_solves(solve, steps, warmup, label):
    """Warm-up, then `steps` timed solves bracketed by device syncs; returns
    (seconds per solve, product ms sum, product launches, last stats)."""
    import torch
    log(f"{label}: warmup {warmup}")
    for _ in range(warmup):
        solve(time_products=False)
    torch.cuda.synchronize()
    log(f"{label}: timing {steps} solves")
    prod_ms, prod_n, last = 0.0, 0, None
    t0 = time.perf_counter()
    for _ in range(steps):
        last = solve(time_products=True)
        st0 = last[0] if isinstance(last, list) else last
        prod_ms += st0["product_ms_sum"]
        prod_n += st0["product_launches"]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, prod_ms, prod_n, last


def bench_single(args, wl, spcg, workloads, torch, dev):
    log(f"generating {args.workload}")
    p = workloads.make_config(wl["cfg"], device=dev, storage=wl["storage"])
    torch.cuda.synchronize()
    N, d = p.N, p.d
    ctx = spcg.Context(0)
    beta = torch.zeros(d, dtype=torch.float64, device=dev)
    W = None
    methods = ["spcg", "pcg"]
    sketch = wl.get("sketch", "srht")
    if sketch == "cs":
        methods = ["spcg", "spcg_srht", "pcg"]
    if args.workload == "learned":
        from paper_2607_25272_amd import schedule
        W = schedule.load_weights(dev)
        methods = ["learned", "spcg", "pcg"]

    def make(method):
        def solve(time_products=False, time_phases=False):
            kw = dict(time_products=time_products, time_phases=time_phases, seed=1, col_scale=p.col_scale,
                      sketch="srht" if method == "spcg_srht" else sketch)
            if method == "learned":
                kw.update(schedule="learned", weights=W)
            _, st = spcg.spcg_solve(ctx, p.X, p.Y, beta=beta, method="pcg" if method == "pcg" else "spcg",
                                    **kw)
            return st
        return solve

    res = {}
    for method in methods:
        solve = make(method)
        dt, pms, pn, last = timed_solves(solve, args.steps, args.warmup, method)
        ph = solve(time_phases=True)
        torch.cuda.synchronize()
        rel = None if args.skip_check else pred_error_vs_ols(p, beta)
        torch.cuda.empty_cache()
        res[method] = dict(s=dt, stats=last, phases=ph, prod_ms=pms, prod_n=pn, rel=rel)
        log(f"{method}: {dt * 1e3:.3f} ms/solve, K={last['K']} T1={last['T_stage1']} T2={last['T_stage2']} "
            f"a={last['policy_a']} stride={last['policy_stride']} syncs={last['host_syncs']} rel={rel} "
            f"phases sketch={ph['t_sketch_ms']:.3f} precond={ph['t_precond_ms']:.3f} "
            f"stage1={ph['t_stage1_ms']:.3f} stage2={ph['t_stage2_ms']:.3f} ms")
    head = "learned" if args.workload == "learned" else "spcg"
    sp, pc = res[head], res["pcg"]
    # roofline of the full-data product (Stage II / full PCG dual pass): one
    # read of X plus the FP64 response vector per launch
    bpl = float(N) * d * p.X.element_size() + float(N) * 8.0
    n_launch = sum(r["prod_n"] for r in res.values())
    avg_ms = sum(r["prod_ms"] for r in res.values()) / max(n_launch, 1)
    rf = roofline(avg_ms, n_launch, bpl, "product_ring_kernel (SG mode, full data)")
    # the same product kernel streams the same X for the CountSketch variants
    rf["traffic"] = SG_TRAFFIC_BYTES.get(wl.get("base", args.workload))
    cpu = None
    if not args.no_cpu_baseline:
        n_s = min(args.cpu_sample, N // 2)
        log(f"cpu baseline: oracle SPCG on {n_s} rows")
        t_cpu, threads = cpu_baseline(p.x_f64(slice(0, n_s)), p.Y, n_s)
        cpu = {"value": t_cpu * N / n_s, "unit": "s", "cores": threads, "kind": "oracle",
               "sample": f"FP64 NumPy oracle SPCG on the first {n_s} rows (d={d}) of the same workload "
                         f"took {t_cpu:.2f} s; value scaled linearly by N/{n_s}"}
    dtype = {"f32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}[wl["storage"]]
    out = {
        "metric": METRIC, "value": sp["s"], "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sp["s"] * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": wl["desc"], "tol": 5e-7, "a_i": sp["stats"]["policy_a"], "r": 6 * d,
                   "m_1": 4 * d, "stage_stride": sp["stats"]["policy_stride"], "K": sp["stats"]["K"],
                   "T_stage1": sp["stats"]["T_stage1"], "T_stage2": sp["stats"]["T_stage2"],
                   "sketch": "CountSketch (SPCG-CS)" if sketch == "cs" else "SRHT"},
        "full_pcg_s": pc["s"], "full_pcg_iters": pc["stats"]["T_stage2"],
        "speedup_vs_full_pcg": pc["s"] / sp["s"],
        "rel_pred_error_vs_ols": {m: res[m]["rel"] for m in res},
        "phases_ms": {m: {k: round(res[m]["phases"][k], 4) for k in
                          ("t_sketch_ms", "t_precond_ms", "t_stage1_ms", "t_stage2_ms", "t_total_ms")}
                      for m in res},
        "host_syncs": {m: res[m]["stats"]["host_syncs"] for m in res},
        "roofline": rf, "cpu_baseline": cpu,
    }
    if sketch == "cs":
        out["spcg_srht_s"] = res["spcg_srht"]["s"]
        out["cs_speedup_vs_srht"] = res["spcg_srht"]["s"] / sp["s"]
    if args.workload == "learned":
        out["plain_schedule_s"] = res["spcg"]["s"]
        out["learned_gain_vs_plain"] = res["spcg"]["s"] / sp["s"]
    ctx.close()
    return out


def bench_batched(args, spcg, workloads, torch, dev):
    log("generating 256 batched problems")
    probs = workloads.batched(device=dev)
    torch.cuda.synchronize()
    Xs, Ys = [q.X for q in probs], [q.Y for q in probs]
    betas = [torch.zeros(q.d, q.k, dtype=torch.float64, device=dev) for q in probs]
    total_bytes = sum(q.N * q.d * 4 for q in probs)
    log(f"{len(probs)} problems, {total_bytes / 1e9:.1f} GB of X, {sum(q.k for q in probs)} right-hand sides")
    ctx = spcg.Context(0)
    res = {}
    for method in ("spcg", "pcg"):
        def solve(time_products=False, time_phases=False, method=method):
            _, st = spcg.spcg_solve_batched(ctx, Xs, Ys, betas=betas, method=method, seed=1,
                                            time_products=time_products, time_phases=time_phases)
            return st
        dt, pms, pn, last = timed_solves(solve, args.steps, args.warmup, method)
        ph = solve(time_phases=True)[0]
        torch.cuda.synchronize()
        rel = None
        if not args.skip_check:
            rel = max(pred_error_vs_ols(q, b) for q, b in zip(probs, betas))
        res[method] = dict(s=dt, stats=last, phases=ph, prod_ms=pms, prod_n=pn,
                           bytes=last[0]["product_bytes"], rel=rel)
        conv = sum(int(s["converged"]) for s in last)
        log(f"{method}: {dt * 1e3:.2f} ms/batch, converged {conv}/{len(probs)}, max rel {rel}, "
            f"phases sketch={ph['t_sketch_ms']:.2f} precond={ph['t_precond_ms']:.2f} "
            f"stage1={ph['t_stage1_ms']:.2f} stage2={ph['t_stage2_ms']:.2f} ms")
    sp, pc = res["spcg"], res["pcg"]
    # the last timed solve of each method gives bytes and launches; the
    # average launch duration comes from every timed solve
    launches_last = sp["stats"][0]["product_launches"] + pc["stats"][0]["product_launches"]
    bpl = (sp["bytes"] + pc["bytes"]) / max(launches_last, 1)
    avg_ms = (sp["prod_ms"] + pc["prod_ms"]) / max(sp["prod_n"] + pc["prod_n"], 1)
    rf = roofline(avg_ms, sp["prod_n"] + pc["prod_n"], bpl, "mrhs_product_kernel (SG mode, full data, MFMA)")
    ctx.close()
    return {
        "metric": METRIC, "value": sp["s"], "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sp["s"] * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOADS["batched"]["desc"], "problems": len(probs),
                   "rhs_total": sum(q.k for q in probs), "x_bytes": total_bytes, "tol": 5e-7, "a_i": 3},
        "full_pcg_s": pc["s"], "speedup_vs_full_pcg": pc["s"] / sp["s"],
        "rel_pred_error_vs_ols": {"spcg": sp["rel"], "pcg": pc["rel"]},
        "phases_ms": {m: {k: round(res[m]["phases"][k], 3) for k in
                          ("t_sketch_ms", "t_precond_ms", "t_stage1_ms", "t_stage2_ms", "t_total_ms")}
                      for m in res},
        "roofline": rf, "cpu_baseline": None,
    }


def bench_paper(args, spcg, workloads, torch, dev):
    """Sec. 4 / Table 1 setting on the GPU: iterations and solve times."""
    rows = []
    ctx = spcg.Context(0)
    for L, kappa in ((17, 1e4), (18, 1e4), (19, 1e4), (20, 1e4), (21, 1e8), (22, 1e8)):
        N = 1 << L
        p = workloads.paper_table1(N, kappa, device=dev)
        beta = torch.zeros(64, dtype=torch.float64, device=dev)
        entry = {"N": N, "kappa": kappa}
        for method in ("spcg", "pcg"):
            kw = dict(beta=beta, seed=1, method=method, m0=8 * 64, m_max=N // 2)
            for _ in range(args.warmup):
                spcg.spcg_solve(ctx, p.X, p.Y, **kw)
            torch.cuda.synchronize()
            ts = []
            for _ in range(args.steps):
                t0 = time.perf_counter()
                _, st = spcg.spcg_solve(ctx, p.X, p.Y, **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            rel = pred_error_vs_ols(p, beta) if not args.skip_check else None
            entry[method] = {"s": statistics.median(ts), "iters": st["T_stage1"] + st["T_stage2"],
                             "K": st["K"], "rel": rel}
        log(f"N=2^{L} kappa={kappa:g}: SPCG {entry['spcg']['iters']} it {entry['spcg']['s'] * 1e3:.2f} ms, "
            f"PCG {entry['pcg']['iters']} it {entry['pcg']['s'] * 1e3:.2f} ms")
        rows.append(entry)
        del p
    ctx.close()
    tot_s = sum(r["spcg"]["s"] for r in rows)
    return {
        "metric": METRIC, "value": tot_s, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": tot_s * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["paper"]["desc"], "value_is": "sum of the six median SPCG times"},
        "rows": rows, "roofline": None, "cpu_baseline": None,
    }


def bench_tuned(args, spcg, workloads, torch, dev):
    """Sec. 4.3 refinements on the GPU: schedules and CountSketch at N=2^22."""
    N, d = 1 << 22, 64
    p = workloads.paper_table1(N, 1e8, device=dev)
    ctx = spcg.Context(0)
    beta = torch.zeros(d, dtype=torch.float64, device=dev)
    tuned = [2 ** k for k in range(10, 17)] + [2 ** 20]
    variants = {
        "spcg": dict(m0=8 * d, m_max=N // 2),
        "spcg_tuned": dict(m_list=tuned, a=4),
        "spcg_theory": dict(m0=8 * d, m_max=N // 2, a_rule="theory", omega=0.5),
        "spcg_cs": dict(m0=8 * d, m_max=N // 2, sketch="cs"),
        "spcg_cs_tuned": dict(m_list=tuned, a=4, sketch="cs"),
        "pcg": dict(method="pcg"),
    }
    res = {}
    for name, kw in variants.items():
        kw = dict(kw, beta=beta, seed=1)
        for _ in range(args.warmup):
            spcg.spcg_solve(ctx, p.X, p.Y, **kw)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            _, st = spcg.spcg_solve(ctx, p.X, p.Y, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        _, ph = spcg.spcg_solve(ctx, p.X, p.Y, time_phases=True, **kw)
        rel = pred_error_vs_ols(p, beta) if not args.skip_check else None
        res[name] = {"s": statistics.median(ts), "K": st["K"], "T_stage1": st["T_stage1"],
                     "T_stage2": st["T_stage2"], "rel": rel,
                     "phases_ms": {k: round(ph[k], 3) for k in ("t_sketch_ms", "t_precond_ms", "t_stage1_ms",
                                                               "t_stage2_ms")}}
        log(f"{name}: {res[name]['s'] * 1e3:.2f} ms, K={st['K']} T1={st['T_stage1']} T2={st['T_stage2']} rel={rel}")
    ctx.close()
    sp = res["spcg"]
    return {
        "metric": METRIC, "value": sp["s"], "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sp["s"] * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["tuned"]["desc"], "value_is": "median SPCG time (paper schedule)"},
        "variants": res, "roofline": None, "cpu_baseline": None,
    }


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
                    help="first run one 1 GiB device-to-device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the row-sharded multi-GPU design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2607_25272_amd as spcg
    import workloads

    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst
    if args.workload == "batched":
        out = bench_batched(args, spcg, workloads, torch, dev)
    elif args.workload == "paper":
        out = bench_paper(args, spcg, workloads, torch, dev)
    elif args.workload == "tuned":
        out = bench_tuned(args, spcg, workloads, torch, dev)
    else:
        out = bench_single(args, WORKLOADS[args.workload], spcg, workloads, torch, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

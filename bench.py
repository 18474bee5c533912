"""Benchmark: time-to-OLS-accuracy of SPCG vs full PCG on one MI355X.

A step is one whole solve (nested sketch, FP64 QR preconditioner, Stage I
sketched PCG stages, Stage II full-data PCG until the stopping test) of a
synthetic least-squares problem already resident in HBM.  Prints one JSON
line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload NAME]

cfg2 (default)  the headline workload: N=4e6, d=1000, X = T C (Student-t(3)
                rows, correlation factor of condition 1e5), sigma=0.5.
                value = SPCG (SRHT) with X stored FP32 (the unquantized
                data); beside it full PCG, SPCG-CS (CountSketch, Sec. 4.3)
                and full PCG with the CountSketch preconditioner, and the
                precision form: the same solves with X stored BF16 and
                FP8-e4m3 (per-column scales), each with its error against
                the OLS estimator of the stored and of the unquantized data
cfg2f32 / cfg2bf16 / cfg2fp8  one storage type of the same problem (SPCG vs full PCG)
cfg1            N=1e6, d=500, FP32 storage
cfg1cs / cfg2cs the same problems solved by SPCG-CS; SPCG-SRHT and full PCG
                are timed beside it
batched         256 independent problems, N in [5e4, 5e5], d in [32, 512],
                1..16 right-hand sides, FP32 (batched / multi-RHS form)
learned         N=2e6, d=256, 1% of rows scaled by 100: plain vs learned schedule
paper           the Sec. 4 / Table 1 setting (d=64, sigma^2=1e-8, m_1=8d,
                m_K=N/2, FP64), N=2^17..2^22: iteration counts and GPU times
tuned           the Sec. 4.3 setting (N=2^22, d=64, kappa=1e8): paper schedule,
                tuned sizes, theory-driven a_i, CountSketch, full PCG

Timing: W untimed warm-up solves, then K timed solves bracketed by device
synchronisations, with no per-launch events in them (every method is timed
the same way).  Per-kernel durations come from separate instrumented solves
of the same workload (time_products = 2: HIP events on the library's stream
around every launch), which also give the roofline figures.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E

T3_DESC = ("X = T C, T Student-t(3), C = Q1 diag(s) Q2^T with s log-spaced 1..1e5; N=4000000, d=1000; "
           "sigma=0.5")
WORKLOADS = {
    "cfg2": dict(cfg=2, storage="f32", headline=True,
                 desc=T3_DESC + "; X stored FP32 (the unquantized data); precision form beside it: "
                                "X stored BF16 and FP8 e4m3 with per-column scales"),
    "cfg2f32": dict(cfg=2, storage="f32", desc=T3_DESC + "; X stored FP32"),
    "cfg2bf16": dict(cfg=2, storage="bf16", desc=T3_DESC + "; X stored BF16"),
    "cfg2fp8": dict(cfg=2, storage="fp8", desc=T3_DESC + "; X stored FP8 e4m3 with per-column scales"),
    "cfg1": dict(cfg=1, storage="f32",
                 desc="X = G diag(s), G Gaussian, s log-spaced 1..1e4; N=1000000, d=500; sigma=1; "
                      "X stored FP32"),
    "cfg1cs": dict(cfg=1, storage="f32", sketch="cs",
                   desc="X = G diag(s), G Gaussian, s log-spaced 1..1e4; N=1000000, d=500; sigma=1; "
                        "X stored FP32; SPCG-CS (nested CountSketch)"),
    "cfg2cs": dict(cfg=2, storage="bf16", sketch="cs",
                   desc=T3_DESC + "; X stored BF16; SPCG-CS (nested CountSketch)"),
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
DTYPE_NAME = {"f32": "f32", "bf16": "bf16", "fp8": "fp8e4m3", "f64": "f64"}

# kernel classes of spcg_solve_stats.kernel_* (include/spcg.h SPCG_KT_*)
KT_NAMES = ["transform_first_pass", "transform_last_pass", "product_S", "product_G", "product_SG",
            "phase_A", "phase_B"]
KT_KERNELS = ["fwht_ring_kernel / fwht_stream_kernel / fwht_pass_kernel (first SRHT pass: gather X[p(k)], "
              "signs, first bits; writes Z)",
              "fwht_ring_kernel / fwht_split_kernel / fwht_stream_kernel / fwht_pass_kernel (last SRHT pass: "
              "remaining bits, "
              "scatter to S_K X and S_hat X)",
              "product_ring_kernel (S mode: s = c2 A^T A p, Stage I)",
              "product_ring_kernel (G mode: stage-start gradient)",
              "product_ring_kernel (SG mode: s and the refreshed gradient, full data)",
              "phase_a_kernel", "phase_b_kernel"]
BYTE_CLASSES = range(5)
# HBM bytes per launch from rocprofv3 PMC runs (2.0 x FETCH_SIZE + WRITE_SIZE,
# calibrated on a 1 GiB copy) for a kernel class and workload, taken on the
# kernel as it now stands; everything else reports null.
_T3_F32 = {"transform_first_pass": 3.4561e10, "transform_last_pass": 2.5994e10, "product_S": 1.6782e9,
           "product_G": 3.3745e9, "product_SG": 1.6036e10}   # profiles/hbm_traffic_t3corr_N4e6_d1000_f32.txt
PMC_TRAFFIC = {(k, w): v for k, v in _T3_F32.items() for w in ("cfg2", "cfg2f32")}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class OlsError:
    """||X (beta - beta_ols)|| / ||X beta|| for one stored matrix, without
    forming beta_ols: with G = X^T X and g = X^T (Y - X beta),
    X^T X (beta_ols - beta) = g, so ||X (beta - beta_ols)||^2 = g^T G^-1 g.
    G is accumulated once in FP64 over row chunks (no library call sees more
    than 2^31 elements) and factored by Cholesky; each beta then costs one
    FP64 pass for g and ||X beta||.  A measurement estimate: the full-size
    comparison against the oracle's TSQR is a test."""

    def __init__(self, X, Y, col_scale=None, chunk=1 << 18):
        import torch
        self.X, self.Y, self.sc, self.chunk = X, Y, col_scale, chunk
        d = X.shape[1]
        G = torch.zeros(d, d, dtype=torch.float64, device=X.device)
        for i in range(0, X.shape[0], chunk):
            xb = self._rows(i)
            G += xb.T @ xb
            del xb
        self.L = torch.linalg.cholesky(G)

    def _rows(self, i):
        import torch
        xb = self.X[i:i + self.chunk].to(torch.float64)
        return xb * self.sc.to(torch.float64) if self.sc is not None else xb

    def __call__(self, beta):
        import torch
        d = self.X.shape[1]
        k = self.Y.shape[1]
        b = beta.reshape(d, k)
        g = torch.zeros(d, k, dtype=torch.float64, device=beta.device)
        fit2 = torch.zeros(k, dtype=torch.float64, device=beta.device)
        for i in range(0, self.X.shape[0], self.chunk):
            xb = self._rows(i)
            f = xb @ b
            g += xb.T @ (self.Y[i:i + self.chunk] - f)
            fit2 += (f * f).sum(0)
            del xb, f
        z = torch.cholesky_solve(g, self.L)
        err = torch.sqrt(torch.clamp((g * z).sum(0), min=0.0)) / torch.sqrt(torch.clamp(fit2, min=1e-300))
        return float(err.max())


def pred_error_vs_ols(p, beta, chunk=1 << 18):
    return OlsError(p.X, p.Y, p.col_scale, chunk)(beta)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return None


def cpu_baseline(Xs, Y, N, gpu_T2, seed=1):
    """The FP64 NumPy oracle's SPCG (oracle.spcg.spcg, as it stands) on the
    first n_s rows of the workload, timed by phase on this host, and the
    phase-by-phase extrapolation of that time to the full N:
    * sketch: the transform costs O(N' log2 N') per column;
    * preconditioner: the QR of the r = 6d rows of S_hat X is the same work;
    * Stage I: proportional to sum_i (a_i + 1) m_i (one gradient pass and a_i
      iterations of two passes over m_i rows per stage);
    * Stage II: proportional to N (2 + 3 T_II) (the oracle's starting
      gradient takes two passes, each iteration three), with T_II the full
      solve's Stage II count measured on the GPU (Algorithm 1 runs the same
      iterations on either)."""
    import numpy as np
    from oracle.spcg import schedule, spcg
    n_s, d = Xs.shape
    Xs = Xs.double().cpu().numpy()
    Ys = Y[:n_s, 0].cpu().numpy()
    t = {}
    t0 = time.perf_counter()
    _, info = spcg(Xs, Ys, seed=seed, timings=t)
    total = time.perf_counter() - t0
    sizes_s, sizes_f = info["sizes"], schedule(N, d)
    T2_s = info["per_rhs"][0]["T"] - info["per_rhs"][0]["T_stage1"]
    Ls, Lf = max(1, (n_s - 1).bit_length()), max(1, (N - 1).bit_length())
    f_sketch = ((1 << Lf) * Lf) / ((1 << Ls) * Ls)
    f_stage1 = sum(4 * m for m in sizes_f) / max(sum(4 * m for m in sizes_s), 1)
    f_stage2 = (N * (2 + 3 * gpu_T2)) / (n_s * (2 + 3 * T2_s))
    est = t["sketch"] * f_sketch + t["precond"] + t["stage1"] * f_stage1 + t["stage2"] * f_stage2
    desc = (f"FP64 NumPy oracle SPCG on the first {n_s} rows (d={d}): K={len(sizes_s)}, T_II={T2_s}, "
            f"{total:.2f} s (sketch {t['sketch']:.2f}, preconditioner {t['precond']:.2f}, Stage I "
            f"{t['stage1']:.2f}, Stage II {t['stage2']:.2f} s); value extrapolated to N={N} (K={len(sizes_f)}, "
            f"T_II={gpu_T2}) phase by phase: sketch x N'log2N' ({f_sketch:.1f}), preconditioner x 1, "
            f"Stage I x sum (a_i+1) m_i ({f_stage1:.1f}), Stage II x N (2 + 3 T_II) ({f_stage2:.1f})")
    return {"value": est, "unit": "s", "cores": blas_threads() or os.cpu_count(), "kind": "oracle",
            "sample": desc, "sample_rows": n_s, "sample_s": total, "sample_phases_s": t,
            "host_cpus": os.cpu_count(), "blas_threads": blas_threads()}


def roofline(kern, cls, workload):
    """The roofline entry of kernel class cls from instrumented solves."""
    k = kern[KT_NAMES[cls]]
    traffic = PMC_TRAFFIC.get((KT_NAMES[cls], workload))
    return {"bound": "hbm", "achieved": k["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": k["GBps"] / HBM_PEAK_GBPS if k["GBps"] else None, "traffic": traffic,
            "kernel": KT_KERNELS[cls], "class": KT_NAMES[cls], "bytes_per_launch": k["bytes_per_launch"],
            "avg_launch_ms": k["avg_ms"], "launches": k["launches"], "ms_per_solve": k["ms_per_solve"]}


def kernel_table(stats_list):
    """Per kernel class over instrumented solves: launches and ms per solve,
    average launch duration, algorithmic bytes per launch, achieved GB/s."""
    n = len(stats_list)
    out = {}
    for c, name in enumerate(KT_NAMES):
        ms = sum(s["kernel_ms"][c] for s in stats_list)
        by = sum(s["kernel_bytes"][c] for s in stats_list)
        nl = sum(s["kernel_launches"][c] for s in stats_list)
        if nl == 0:
            continue
        out[name] = {"launches_per_solve": nl / n, "ms_per_solve": ms / n, "avg_ms": ms / nl,
                     "bytes_per_launch": by / nl if c in BYTE_CLASSES else None,
                     "GBps": (by / (ms * 1e-3) / 1e9) if (c in BYTE_CLASSES and ms > 0) else None,
                     "launches": nl}
        if out[name]["GBps"] is not None:
            out[name]["frac"] = out[name]["GBps"] / HBM_PEAK_GBPS
    return out


def dominant_class(kern):
    best, cls = -1.0, None
    for c in BYTE_CLASSES:
        k = kern.get(KT_NAMES[c])
        if k and k["ms_per_solve"] > best:
            best, cls = k["ms_per_solve"], c
    return cls


def measure(solve, steps, warmup, label, instrumented=2):
    """W warm-up solves, K timed solves (device syncs around the loop, no
    per-launch events), one solve with phase times, then `instrumented`
    solves with every launch timed by kernel class."""
    import torch
    log(f"{label}: warmup {warmup}")
    for _ in range(warmup):
        solve()
    torch.cuda.synchronize()
    log(f"{label}: timing {steps} solves")
    t0 = time.perf_counter()
    for _ in range(steps):
        last = solve()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ph = solve(time_phases=True)
    inst = [solve(time_products=2) for _ in range(instrumented)]
    torch.cuda.synchronize()
    kern = kernel_table(inst) if instrumented else {}
    log(f"{label}: {dt * 1e3:.3f} ms/solve, K={last['K']} T1={last['T_stage1']} T2={last['T_stage2']} "
        f"a={last['policy_a']} stride={last['policy_stride']} syncs={last['host_syncs']} "
        f"phases sketch={ph['t_sketch_ms']:.3f} precond={ph['t_precond_ms']:.3f} "
        f"stage1={ph['t_stage1_ms']:.3f} stage2={ph['t_stage2_ms']:.3f} ms")
    for name, k in kern.items():
        gb = f"{k['GBps']:.0f} GB/s" if k.get("GBps") else "-"
        log(f"{label}:   {name}: {k['launches_per_solve']:.1f} launches, {k['ms_per_solve']:.3f} ms/solve, "
            f"{k['avg_ms'] * 1e3:.1f} us avg, {gb}")
    return {"s": dt, "stats": last, "phases": ph, "kernels": kern}


def phases_dict(ph):
    return {k: round(ph[k], 4) for k in ("t_sketch_ms", "t_precond_ms", "t_stage1_ms", "t_stage2_ms",
                                          "t_total_ms")}


def solver(spcg, ctx, X, Y, col_scale, beta, method, sketch, extra=None):
    def solve(time_products=0, time_phases=False):
        kw = dict(time_products=time_products, time_phases=time_phases, seed=1, col_scale=col_scale,
                  sketch=sketch)
        if extra:
            kw.update(extra)
        _, st = spcg.spcg_solve(ctx, X, Y, beta=beta, method=method, **kw)
        return st
    return solve


TUNED_SIZES = [1 << k for k in range(10, 17)] + [1 << 20]   # Sec. 4.3: 2^10 .. 2^16, then 2^20


def learned_weights(dev):
    """The shipped per-stage schedule network, or None if it is missing."""
    from paper_2607_25272_amd import schedule
    try:
        return schedule.load_weights(dev)
    except (OSError, ValueError) as e:
        log(f"no learned schedule weights: {e}")
        return None


def solve_cost_fn(spcg, ctx, X, Y, sc, sketch):
    """Bytes read by a solve's product passes (schedule.solve_cost) from its
    stats; the stage sizes are those of the default sketch of (X, Y)."""
    import torch
    from paper_2607_25272_amd import schedule
    sk = spcg.spcg_sketch(ctx, X, Y, seed=1, col_scale=sc, kind=sketch)
    sizes = list(sk.sizes)
    A, _, _ = sk.view(len(sizes) - 1)
    e_b = {spcg.SPCG_F64: 8, spcg.SPCG_F32: 4, spcg.SPCG_BF16: 2}[A.dtype]
    sk.free()
    e_x = {torch.float64: 8, torch.float32: 4, torch.bfloat16: 2, torch.float8_e4m3fn: 1}[X.dtype]
    N, d = X.shape

    def cost(st, run_sizes=None):
        sz = sizes if run_sizes is None else run_sizes
        if st["stages_planned"] != len(sz):
            return None
        return schedule.solve_cost(st, sz, N, d, e_x, e_b, nested=sketch == "srht")
    return cost


def bench_headline(args, wl, spcg, workloads, torch, dev):
    """N=4e6, d=1000: SPCG vs full PCG with both sketch kinds on the FP32
    (unquantized) data, and the precision form in BF16 and FP8."""
    log("generating cfg2 (FP32 = unquantized) and its BF16 / FP8 copies")
    p = workloads.make_config(2, device=dev, storage="f32")
    stores = {"f32": (p.X, None), "bf16": workloads.store(p.X, "bf16"), "fp8": workloads.store(p.X, "fp8")}
    torch.cuda.synchronize()
    N, d = p.N, p.d
    ctx = spcg.Context(0)
    beta = torch.zeros(d, dtype=torch.float64, device=dev)
    log("FP64 Gram of the unquantized data")
    err_unq = OlsError(p.X, p.Y)
    runs = {}
    plan = [("f32", "srht"), ("f32", "cs"), ("bf16", "srht"), ("fp8", "srht"), ("bf16", "cs"), ("fp8", "cs")]
    W = learned_weights(dev)
    # beside Algorithm 1 as written (a_i = 3, every prefix): the learned
    # per-stage schedule and the Sec. 4.3 tuned sizes, with the SRHT
    extra = {"learned": ("spcg", dict(schedule="learned", weights=W)) if W is not None else None,
             "tuned": ("spcg", dict(m_list=TUNED_SIZES, a=4))}
    costs = {}
    for storage, sk in plan:
        X, sc = stores[storage]
        err_st = err_unq if storage == "f32" else OlsError(X, p.Y, sc)
        cost = solve_cost_fn(spcg, ctx, X, p.Y, sc, sk)
        methods = [("spcg", "spcg", None), ("pcg", "pcg", None)]
        if sk == "srht":
            methods += [(k, v[0], v[1]) for k, v in extra.items() if v is not None]
        for mname, method, kw in methods:
            name = f"{storage}_{sk}_{mname}"
            r = measure(solver(spcg, ctx, X, p.Y, sc, beta, method, sk, kw), args.steps, args.warmup, name,
                        instrumented=2 if storage == "f32" or method == "spcg" else 1)
            costs[name] = cost(r["stats"], TUNED_SIZES if mname == "tuned" else None)
            if not args.skip_check:
                r["rel"] = err_st(beta)
                r["rel_unquantized"] = err_unq(beta) if storage != "f32" else r["rel"]
                log(f"{name}: rel vs OLS of the stored data {r['rel']:.3e}, of the unquantized data "
                    f"{r['rel_unquantized']:.3e}")
            runs[name] = r
        del err_st
        torch.cuda.empty_cache()
    head = runs["f32_srht_spcg"]
    kern = head["kernels"]
    dom = dominant_class(kern)
    rf = roofline(kern, dom, "cfg2")
    rf["workload"] = "SPCG (SRHT) step at N=4e6, d=1000, FP32"
    cpu = None
    if not args.no_cpu_baseline:
        n_s = min(args.cpu_sample or 131072, N // 2)
        log(f"cpu baseline: oracle SPCG on {n_s} rows")
        cpu = cpu_baseline(p.X[:n_s], p.Y, N, head["stats"]["T_stage2"])
        log(f"cpu baseline: {cpu['sample']}")

    def line(r):
        st = r["stats"]
        out = {"s": r["s"], "K": st["K"], "T_stage1": st["T_stage1"], "T_stage2": st["T_stage2"],
               "host_syncs": st["host_syncs"], "phases_ms": phases_dict(r["phases"])}
        if "rel" in r:
            out["rel_vs_ols_stored"] = r["rel"]
            out["rel_vs_ols_unquantized"] = r["rel_unquantized"]
        return out

    solves = {name: line(r) for name, r in runs.items()}
    for name in solves:
        solves[name]["product_bytes_read"] = costs[name]
    schedules = {}
    for storage in ("f32", "bf16", "fp8"):
        base = f"{storage}_srht_spcg"
        for k in ("learned", "tuned"):
            name = f"{storage}_srht_{k}"
            if name in runs:
                schedules[name] = {"time_plain_over_this": runs[base]["s"] / runs[name]["s"],
                                   "bytes_plain_over_this": (costs[base] / costs[name]
                                                             if costs[base] and costs[name] else None),
                                   "stage_iters": runs[name]["stats"]["stage_iters"][
                                       :runs[name]["stats"]["stages_planned"]],
                                   "vs_full_pcg": runs[f"{storage}_srht_pcg"]["s"] / runs[name]["s"]}
    speedups = {f"{s}_{k}": runs[f"{s}_{k}_pcg"]["s"] / runs[f"{s}_{k}_spcg"]["s"] for s, k in plan}
    kernels = {name: r["kernels"] for name, r in runs.items() if name.endswith("_spcg") or name.startswith("f32")}
    out = {
        "metric": METRIC, "value": head["s"], "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["s"] * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["desc"], "N": N, "d": d, "tol": 5e-7, "a_i": head["stats"]["policy_a"],
                   "r": 6 * d, "m_1": 4 * d, "K": head["stats"]["K"], "T_stage1": head["stats"]["T_stage1"],
                   "T_stage2": head["stats"]["T_stage2"], "sketch": "SRHT", "value_is": "SPCG (SRHT), X FP32"},
        "full_pcg_s": runs["f32_srht_pcg"]["s"], "full_pcg_iters": runs["f32_srht_pcg"]["stats"]["T_stage2"],
        "speedup_vs_full_pcg": speedups["f32_srht"],
        "rel_pred_error_vs_ols": {"spcg": head.get("rel"), "pcg": runs["f32_srht_pcg"].get("rel")},
        "speedups_vs_full_pcg_same_sketch": speedups,
        "schedules_vs_plain": schedules,
        "solves": solves,
        "roofline": rf, "kernels": kernels, "cpu_baseline": cpu,
    }
    ctx.close()
    return out


def bench_single(args, wl, spcg, workloads, torch, dev):
    log(f"generating {args.workload}")
    p = workloads.make_config(wl["cfg"], device=dev, storage=wl["storage"])
    torch.cuda.synchronize()
    N, d = p.N, p.d
    ctx = spcg.Context(0)
    beta = torch.zeros(d, dtype=torch.float64, device=dev)
    sketch = wl.get("sketch", "srht")
    methods = [("spcg", "spcg", sketch, None), ("pcg", "pcg", sketch, None)]
    if sketch == "cs":
        methods.insert(1, ("spcg_srht", "spcg", "srht", None))
        methods.append(("pcg_srht", "pcg", "srht", None))
    if args.workload == "learned":
        from paper_2607_25272_amd import schedule
        W = schedule.load_weights(dev)
        methods.insert(0, ("learned", "spcg", sketch, dict(schedule="learned", weights=W)))
    err = None if args.skip_check else OlsError(p.X, p.Y, p.col_scale)
    res = {}
    for name, method, sk, extra in methods:
        r = measure(solver(spcg, ctx, p.X, p.Y, p.col_scale, beta, method, sk, extra), args.steps, args.warmup,
                    name)
        r["rel"] = err(beta) if err else None
        res[name] = r
    head = "learned" if args.workload == "learned" else "spcg"
    sp, pc = res[head], res["pcg"]
    dom = dominant_class(sp["kernels"])
    rf = roofline(sp["kernels"], dom, args.workload)
    cpu = None
    if not args.no_cpu_baseline:
        n_s = min(args.cpu_sample or 65536, N // 2)
        log(f"cpu baseline: oracle SPCG on {n_s} rows")
        cpu = cpu_baseline(p.x_f64(slice(0, n_s)), p.Y, N, sp["stats"]["T_stage2"])
    out = {
        "metric": METRIC, "value": sp["s"], "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sp["s"] * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE_NAME[wl["storage"]], "data": "synthetic",
        "config": {"workload": wl["desc"], "tol": 5e-7, "a_i": sp["stats"]["policy_a"], "r": 6 * d,
                   "m_1": 4 * d, "stage_stride": sp["stats"]["policy_stride"], "K": sp["stats"]["K"],
                   "T_stage1": sp["stats"]["T_stage1"], "T_stage2": sp["stats"]["T_stage2"],
                   "sketch": "CountSketch (SPCG-CS)" if sketch == "cs" else "SRHT"},
        "full_pcg_s": pc["s"], "full_pcg_iters": pc["stats"]["T_stage2"],
        "speedup_vs_full_pcg": pc["s"] / sp["s"],
        "rel_pred_error_vs_ols": {m: res[m]["rel"] for m in res},
        "phases_ms": {m: phases_dict(res[m]["phases"]) for m in res},
        "host_syncs": {m: res[m]["stats"]["host_syncs"] for m in res},
        "roofline": rf, "kernels": {m: res[m]["kernels"] for m in res}, "cpu_baseline": cpu,
    }
    if sketch == "cs":
        out["spcg_srht_s"] = res["spcg_srht"]["s"]
        out["pcg_srht_s"] = res["pcg_srht"]["s"]
        out["cs_speedup_vs_srht"] = res["spcg_srht"]["s"] / sp["s"]
    if args.workload == "learned":
        cost = solve_cost_fn(spcg, ctx, p.X, p.Y, p.col_scale, sketch)
        cp, cl = cost(res["spcg"]["stats"]), cost(sp["stats"])
        out["plain_schedule_s"] = res["spcg"]["s"]
        out["learned_gain_vs_plain"] = res["spcg"]["s"] / sp["s"]
        out["learned_bytes_plain_over_learned"] = cp / cl if cp and cl else None
        out["learned_stage_iters"] = sp["stats"]["stage_iters"][:sp["stats"]["stages_planned"]]
    ctx.close()
    return out


def timed_solves(solve, steps, warmup, label):
    """Warm-up, then `steps` timed solves bracketed by device syncs (no
    per-launch events); returns (seconds per solve, 0, 0, last stats)."""
    import torch
    log(f"{label}: warmup {warmup}")
    for _ in range(warmup):
        solve()
    torch.cuda.synchronize()
    log(f"{label}: timing {steps} solves")
    t0 = time.perf_counter()
    for _ in range(steps):
        last = solve()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, 0.0, 0, last


def bench_batched(args, spcg, workloads, torch, dev):
    log("generating 256 batched problems")
    probs = workloads.batched(device=dev)
    torch.cuda.synchronize()
    Xs, Ys = [q.X for q in probs], [q.Y for q in probs]
    betas = [torch.zeros(q.d, q.k, dtype=torch.float64, device=dev) for q in probs]
    total_bytes = sum(q.N * q.d * 4 for q in probs)
    log(f"{len(probs)} problems, {total_bytes / 1e9:.1f} GB of X, {sum(q.k for q in probs)} right-hand sides")
    ctx = spcg.Context(0)
    # the context's first solve tunes the task granularity and the tile
    # shape of every launch bucket (row-width class x k range)
    _, st0 = spcg.spcg_solve_batched(ctx, Xs, Ys, betas=betas, method="spcg", seed=1)
    tuned_shapes = {str(b): v for b, v in enumerate(st0[0]["batch_shapes"]) if v}
    tune_ms = {f"{b // 4}:{b % 4 + 1}": round(v, 3) for b, v in enumerate(st0[0]["batch_tune_ms"]) if v > 0}
    log(f"tuned: {st0[0]['batch_tasks_per_cu']} tasks per CU, shapes per bucket {tuned_shapes}")
    res = {}
    for method in ("spcg", "pcg"):
        def solve(time_products=False, time_phases=False, method=method):
            _, st = spcg.spcg_solve_batched(ctx, Xs, Ys, betas=betas, method=method, seed=1,
                                            time_products=time_products, time_phases=time_phases)
            return st
        dt, pms, pn, last = timed_solves(solve, args.steps, args.warmup, method)
        ph = solve(time_phases=True)[0]
        last = solve(time_products=True)
        torch.cuda.synchronize()
        pms, pn = last[0]["product_ms_sum"], last[0]["product_launches"]
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
    achieved = bpl / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    rf = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
          "frac": achieved / HBM_PEAK_GBPS if achieved else None, "traffic": None,
          "kernel": "mrhs_product_kernel (SG mode, full data, MFMA)", "bytes_per_launch": bpl,
          "avg_launch_ms": avg_ms, "launches": sp["prod_n"] + pc["prod_n"]}
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
        "autotune": {"tasks_per_cu": st0[0]["batch_tasks_per_cu"],
                     "shape_per_bucket": tuned_shapes,
                     "bucket_shape_ms": tune_ms,
                     "buckets": "row-width class * 2 + (k > 8); classes 16x1 16x2 4x1 4x2 4x4 4x8 generic",
                     "shapes": "1 three barriers per tile, 2 two-tile pipeline (3 slots), 3 pipeline (4 slots)"},
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="rows of the oracle's CPU sample (0: 131072 for the d=1000 headline, else 65536)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle on the whole problem (checks the CPU extrapolation; slow)")
    ap.add_argument("--skip-check", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one 1 GiB device-to-device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path has no multi-GPU form)", file=sys.stderr)
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
    wl = WORKLOADS[args.workload]
    if args.workload == "batched":
        out = bench_batched(args, spcg, workloads, torch, dev)
    elif args.workload == "paper":
        out = bench_paper(args, spcg, workloads, torch, dev)
    elif args.workload == "tuned":
        out = bench_tuned(args, spcg, workloads, torch, dev)
    elif wl.get("headline"):
        out = bench_headline(args, wl, spcg, workloads, torch, dev)
    else:
        out = bench_single(args, wl, spcg, workloads, torch, dev)
    if args.cpu_full and args.workload not in ("batched", "paper", "tuned"):
        out["cpu_full_check"] = cpu_full(args, wl, workloads, torch, dev, out)
    print(json.dumps(out), flush=True)


def cpu_full(args, wl, workloads, torch, dev, out):
    """The oracle on the whole problem, to check the extrapolated cpu_baseline."""
    from oracle.spcg import spcg as oracle_spcg
    p = workloads.make_config(wl["cfg"], device=dev, storage=wl["storage"])
    X = p.x_f64().cpu().numpy()
    Y = p.Y[:, 0].cpu().numpy()
    del p
    torch.cuda.empty_cache()
    log(f"cpu full: oracle SPCG on all {X.shape[0]} rows")
    t = {}
    t0 = time.perf_counter()
    _, info = oracle_spcg(X, Y, seed=1, timings=t)
    total = time.perf_counter() - t0
    est = out["cpu_baseline"]["value"] if out.get("cpu_baseline") else None
    log(f"cpu full: {total:.1f} s (extrapolated {est})")
    return {"s": total, "phases_s": t, "T": info["per_rhs"][0]["T"], "extrapolated_s": est,
            "blas_threads": blas_threads(), "host_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()

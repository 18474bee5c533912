"""Trains the learned schedule on the GPU from the method's own runs.

    python -m paper_2607_25272_amd.train_schedule --problems 1250 --out weights.json

For each training problem (``workloads.schedule_training_problem``) the
eight (a, stride) variants are solved with the plain stopping test
(1250 problems give 10,000 labelled runs); the network is then trained by
the library's kernels, and the variants chosen on held-out problems are
scored against the plain schedule (a = 3, stride 1) with the recorded
times.  Writes the weights (JSON) and the labelled data (NPZ).
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(f"[train_schedule] {msg}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--problems", type=int, default=1250)
    ap.add_argument("--holdout", type=float, default=0.1)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="schedule_weights.json")
    ap.add_argument("--data", default=None, help="NPZ of labelled runs to write (or to reuse if it exists)")
    args = ap.parse_args()

    import paper_2607_25272_amd as spcg
    import workloads
    from paper_2607_25272_amd import schedule

    dev = torch.device("cuda", 0)
    ctx = spcg.Context(0)
    records = []
    if args.data and os.path.exists(args.data):
        z = np.load(args.data)
        records = json.loads(str(z["records"]))
        log(f"reusing {len(records)} problems from {args.data}")
    else:
        t0 = time.time()
        for i in range(args.problems):
            p = workloads.schedule_training_problem(i, device=dev)
            runs = schedule.run_variants(ctx, p)
            records.append({"i": i, "N": p.N, "d": p.d, "cond": p.meta["cond"], "rows": p.meta["rows"],
                            "sigma": p.meta["sigma"], "runs": runs})
            del p
            if (i + 1) % 50 == 0 or i + 1 == args.problems:
                log(f"{i + 1}/{args.problems} problems labelled ({time.time() - t0:.1f} s)")
        if args.data:
            np.savez_compressed(args.data, records=np.array(json.dumps(records)))
    n_runs = sum(1 for r in records for v in r["runs"] if "error" not in v)
    log(f"{n_runs} successful runs")

    rng = np.random.default_rng(args.seed)
    order = rng.permutation(len(records))
    n_hold = int(round(args.holdout * len(records)))
    hold = set(order[:n_hold].tolist())
    train_s, hold_recs = [], []
    for j, r in enumerate(records):
        pre, ii = schedule.samples_from_runs(r["runs"])
        if pre is None:
            continue
        if j in hold:
            hold_recs.append(r)
        else:
            train_s.append(pre)
            train_s.extend(ii)
    data = schedule.to_tensors(train_s, dev)
    log(f"training on {len(train_s)} samples")
    W, losses = schedule.train(ctx, data, steps=args.steps, lr=args.lr, seed=args.seed, log=log)

    # held-out evaluation with the recorded times
    tot_plain = tot_learn = tot_best = 0.0
    hits = 0
    s_err = []
    for r in hold_recs:
        runs = {(v["a"], v["stride"]): v for v in r["runs"] if "error" not in v and v["converged"]}
        if schedule.PLAIN not in runs:
            continue
        f = torch.tensor([runs[schedule.PLAIN]["f_pre"]], dtype=torch.float32, device=dev)
        a, st, _ = schedule.predict(ctx, W, f)
        choice = (int(a[0]), int(st[0]))
        best = min(runs.values(), key=lambda v: v["t_ms"])
        hits += int(choice == (best["a"], best["stride"]))
        chosen = runs.get(choice, runs[schedule.PLAIN])
        tot_plain += runs[schedule.PLAIN]["t_ms"]
        tot_learn += chosen["t_ms"]
        tot_best += best["t_ms"]
        fi = torch.tensor([v["f_ii"] for v in runs.values()], dtype=torch.float32, device=dev)
        _, _, s_hat = schedule.predict(ctx, W, fi)
        s_err.extend((np.rint(s_hat) - np.array([v["T2"] for v in runs.values()])).tolist())
    s_err = np.array(s_err)
    evaluation = {
        "holdout_problems": len(hold_recs),
        "policy_match_rate": hits / max(len(hold_recs), 1),
        "recorded_time_ms": {"plain": tot_plain, "learned_choice": tot_learn, "best_variant": tot_best},
        "stage2_count_error": {"mean_abs": float(np.abs(s_err).mean()) if s_err.size else None,
                               "over_by_2_or_more": float((s_err >= 2).mean()) if s_err.size else None},
    }
    log(f"held-out: {json.dumps(evaluation)}")
    meta = {"problems": len(records), "runs": n_runs, "train_samples": len(train_s), "steps": args.steps,
            "lr": args.lr, "seed": args.seed, "final_loss": losses[-1][1], "losses": losses,
            "evaluation": evaluation}
    schedule.save_weights(W, args.out, meta)
    log(f"wrote {args.out}")
    ctx.close()


if __name__ == "__main__":
    main()

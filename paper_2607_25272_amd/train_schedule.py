"""Trains the learned schedule on the GPU from the method's own runs.

    python -m paper_2607_25272_amd.train_schedule --problems 400 --out weights.json --data runs.npz

For each training problem (``workloads.schedule_training_problem``, FP32,
BF16 or FP8 storage) the schedule variants of ``schedule.VARIANTS`` are
solved with the plain stopping test (about 22 runs per problem, so 500
problems give about 10,000 labelled runs); the network is then trained by
the library's kernels.  On held-out problems the learned solve (per-stage
decisions on the device) is compared with the plain schedule (a_i = 3,
every prefix) by the bytes its product passes read and by time.  Writes the
weights (JSON) and the labelled data (NPZ).
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
    ap.add_argument("--problems", type=int, default=500)
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
            p = workloads.schedule_training_problem(i, device=dev, storage="mix")
            sizes, e_x, e_b, runs = schedule.run_variants(ctx, p)
            records.append({"i": i, "N": p.N, "d": p.d, "cond": p.meta["cond"], "rows": p.meta["rows"],
                            "sigma": p.meta["sigma"], "storage": p.meta["storage"], "sizes": sizes,
                            "e_x": e_x, "e_b": e_b, "runs": runs})
            del p
            if (i + 1) % 25 == 0 or i + 1 == args.problems:
                log(f"{i + 1}/{args.problems} problems labelled ({time.time() - t0:.1f} s)")
        if args.data:
            np.savez_compressed(args.data, records=np.array(json.dumps(records)))
    n_runs = sum(1 for r in records for v in r["runs"] if "error" not in v)
    log(f"{n_runs} successful runs")

    # problems split three ways: held out for the final evaluation, a
    # validation part for early stopping, the rest for the gradient
    rng = np.random.default_rng(args.seed)
    order = rng.permutation(len(records))
    n_hold = int(round(args.holdout * len(records)))
    hold = set(order[:n_hold].tolist())
    valid = set(order[n_hold:2 * n_hold].tolist())
    train_s, val_s, hold_recs = [], [], []
    for j, r in enumerate(records):
        stage, ii = schedule.samples_from_runs(r["runs"])
        if not stage:
            continue
        if j in hold:
            hold_recs.append(r)
        elif j in valid:
            val_s.extend(stage)
            val_s.extend(ii)
        else:
            train_s.extend(stage)
            train_s.extend(ii)
    data = schedule.to_tensors(train_s, dev)
    val = schedule.to_tensors(val_s, dev) if val_s else None
    log(f"training on {len(train_s)} samples, validation {len(val_s)}")
    W, losses = schedule.train(ctx, data, steps=args.steps, lr=args.lr, seed=args.seed, log=log, val=val,
                               log_every=100)

    # held-out problems: learned solve against the plain schedule
    tot = {"plain_cost": 0.0, "learned_cost": 0.0, "best_variant_cost": 0.0, "plain_ms": 0.0, "learned_ms": 0.0}
    n_eval = conv = 0
    for r in hold_recs:
        p = workloads.schedule_training_problem(r["i"], device=dev, storage="mix")
        beta = torch.zeros(p.d, dtype=torch.float64, device=dev)
        kw = dict(beta=beta, col_scale=p.col_scale, seed=1, time_phases=True)
        spcg.spcg_solve(ctx, p.X, p.Y, **kw)
        _, sp = spcg.spcg_solve(ctx, p.X, p.Y, **kw)
        spcg.spcg_solve(ctx, p.X, p.Y, schedule="learned", weights=W, **kw)
        _, sl = spcg.spcg_solve(ctx, p.X, p.Y, schedule="learned", weights=W, **kw)
        ok = [v for v in r["runs"] if "error" not in v and v["converged"]]
        if not (sp["converged"] and ok):
            continue
        n_eval += 1
        conv += int(sl["converged"])
        tot["plain_cost"] += schedule.solve_cost(sp, r["sizes"], p.N, p.d, r["e_x"], r["e_b"])
        tot["learned_cost"] += schedule.solve_cost(sl, r["sizes"], p.N, p.d, r["e_x"], r["e_b"])
        tot["best_variant_cost"] += min(v["cost"] for v in ok)
        tot["plain_ms"] += sp["t_total_ms"]
        tot["learned_ms"] += sl["t_total_ms"]
        del p
    evaluation = {"holdout_problems": n_eval, "learned_converged": conv, "totals": tot,
                  "cost_ratio_plain_over_learned": tot["plain_cost"] / max(tot["learned_cost"], 1.0),
                  "time_ratio_plain_over_learned": tot["plain_ms"] / max(tot["learned_ms"], 1e-9)}
    log(f"held-out: {json.dumps(evaluation)}")
    meta = {"problems": len(records), "runs": n_runs, "train_samples": len(train_s),
            "validation_samples": len(val_s), "steps": args.steps, "lr": args.lr, "seed": args.seed,
            "final_loss": losses[-1][1], "losses": losses,
            "evaluation": evaluation}
    schedule.save_weights(W, args.out, meta)
    log(f"wrote {args.out}")
    ctx.close()


if __name__ == "__main__":
    main()

"""Learned schedule: weights, labels from the method's own runs, training.

The network (three dense FP32 layers, see ``include/spcg.h``) decides, at
the start of every sketched stage and on the device, the stage's PCG
iteration count a_i in 0..4 and whether Stage I stops after the stage; at
the start of Stage II it predicts the number of Stage II iterations to run
before the first stopping test.  Everything here runs through the library:
the labels come from ``spcg_solve`` runs with the plain schedule, and
training calls the library's forward/backward and Adam kernels
(``spcg_mlp_loss_grad``, ``spcg_mlp_adam``) on the GPU.

Labels.  For a problem, the variants (a, pattern, j) are solved with the
plain stopping test: every planned stage (every prefix of the sketch) but
the last j runs a_i = a iterations ("all"), a and 0 alternately, ending
with a at the last stage run ("alt"), or a on the first half and on the
last stage run with 0 between ("ends").  Each run is costed by the bytes its
product passes read (``solve_cost``).  Among the converged variants within
2% of the cheapest, the label variant is the one that stops earliest
(largest j), then "all" before "ends" before "alt", then the largest a -- a fixed
tie-break, so that near-equal variants do not scatter the labels.  It
gives one sample per stage it ran (the stage features recorded in that
run, label a_i, stop = 1 at its last stage when j > 0), and every
converged variant gives a Stage II sample (its Stage II features, the
Stage II iteration count the plain test chose).
"""
import json
import os

import numpy as np
import torch

from . import _lib as L
from . import spcg_mlp_adam, spcg_mlp_forward, spcg_mlp_loss_grad, spcg_sketch, spcg_solve

WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedule_weights.json")
NA = L.SPCG_MLP_O - 3          # a_i choices 0..NA-1
VARIANTS = ([(a, "all", j) for a in (2, 3, 4) for j in range(6)]
            + [(4, "alt", j) for j in range(4)]
            + [(a, "ends", j) for a in (3, 4) for j in range(5)])
PATTERN_ORDER = {"all": 2, "ends": 1, "alt": 0}   # label tie-break among near-equal variants
COST_TOL = 1.02
PLAIN = (3, "all", 0)
_ES = {torch.float64: 8, torch.float32: 4, torch.bfloat16: 2, torch.float8_e4m3fn: 1}


def load_weights(device, path=WEIGHTS_PATH):
    """Trained parameters as a float32 device tensor (SPCG_MLP_PARAMS entries)."""
    with open(path) as f:
        blob = json.load(f)
    w = np.asarray(blob["params"], dtype=np.float32)
    if w.size != L.SPCG_MLP_PARAMS or (blob["F"], blob["H"], blob["O"]) != (L.SPCG_MLP_F, L.SPCG_MLP_H,
                                                                          L.SPCG_MLP_O):
        raise ValueError(f"{path}: parameter layout does not match the library")
    return torch.from_numpy(w).to(device)


def save_weights(W, path, meta):
    w = W.detach().float().cpu().numpy()
    blob = {"F": L.SPCG_MLP_F, "H": L.SPCG_MLP_H, "O": L.SPCG_MLP_O, "meta": meta,
            "params": [float(np.format_float_scientific(x, precision=8)) for x in w]}
    with open(path, "w") as f:
        json.dump(blob, f)


def init_weights(seed, device):
    """He initialisation of the weight matrices, zero biases."""
    rng = np.random.default_rng(seed)
    F, H, O = L.SPCG_MLP_F, L.SPCG_MLP_H, L.SPCG_MLP_O
    parts = []
    for shape in ((H, F), (H,), (H, H), (H,), (O, H), (O,)):
        if len(shape) == 2:
            parts.append(rng.standard_normal(shape).ravel() * np.sqrt(2.0 / shape[1]))
        else:
            parts.append(np.zeros(shape))
    return torch.from_numpy(np.concatenate(parts).astype(np.float32)).to(device)


def a_list_of(K, a, pattern, j):
    """Per-stage iteration counts of variant (a, pattern, j) over K planned
    stages: "all" a everywhere, "alt" a and 0 alternately ending with a,
    "ends" a on the first half and on the last stage run, 0 in between (the
    shape of the Sec. 4.3 tuned schedule: small sizes, then one large)."""
    n = K - j
    if pattern == "all":
        return [a] * n
    if pattern == "ends":
        h = (n + 1) // 2
        return [a if (i < h or i == n - 1) else 0 for i in range(n)]
    return [a if (n - 1 - i) % 2 == 0 else 0 for i in range(n)]


def solve_cost(st, sizes, N, d, e_x, e_b, nested=True):
    """Bytes read by the product passes of a solve (deterministic, from its
    stats): Stage I iterations a_i m_i d e_b; the stage-start gradient
    passes m (d e_b + 8) over the rows each start reads (the new rows of a
    nested prefix, else all m_i); Stage II (1 + T_II) N (d e_x + 8)."""
    cost, m_prev = 0.0, 0
    for i, a in enumerate(st["stage_iters"][:st["stages_planned"]]):
        if a < 0:
            continue
        m = sizes[i]
        cost += a * m * d * e_b + (m - (m_prev if nested else 0)) * (d * e_b + 8)
        m_prev = m
    return cost + (1 + st["T_stage2"]) * N * (d * e_x + 8)


def problem_sizes(ctx, prob, seed=1):
    """Planned stage sizes and the stored row element sizes of a problem."""
    sk = spcg_sketch(ctx, prob.X, prob.Y, seed=seed, col_scale=prob.col_scale)
    sizes = list(sk.sizes)
    A, _, _ = sk.view_tensor(len(sizes) - 1) if sizes else (prob.X, None, None)
    e_b = _ES[A.dtype]
    sk.free()
    return sizes, _ES[prob.X.dtype], e_b


def run_variants(ctx, prob, tol=5e-7, seed=1, beta=None):
    """Solves prob with every variant under the plain test.  Returns
    (sizes, e_x, e_b, list of dicts; entries with "error" for failures)."""
    if beta is None:
        beta = torch.zeros(prob.d, dtype=torch.float64, device=prob.X.device)
    sizes, e_x, e_b = problem_sizes(ctx, prob, seed)
    K = len(sizes)
    kw = dict(beta=beta, col_scale=prob.col_scale, seed=seed, tol=tol, record_features=True,
              time_phases=True)
    spcg_solve(ctx, prob.X, prob.Y, **kw)  # workspaces sized, caches warm
    out = []
    for a, pat, j in VARIANTS:
        if j >= K or (pat != "all" and K - j < 3):
            continue
        al = a_list_of(K, a, pat, j)
        try:
            _, st = spcg_solve(ctx, prob.X, prob.Y, a_list=al, stage_limit=K - j, **kw)
        except Exception as e:  # a failing variant gives no label
            out.append({"a": a, "pattern": pat, "j": j, "error": str(e)})
            continue
        n = min(K - j, 16)
        out.append({"a": a, "pattern": pat, "j": j, "a_list": al, "t_ms": st["t_total_ms"],
                    "cost": solve_cost(st, sizes, prob.N, prob.d, e_x, e_b), "T1": st["T_stage1"],
                    "T2": st["T_stage2"], "K": K, "converged": bool(st["converged"]),
                    "syncs": st["host_syncs"], "f_stage": [list(st["stage_features"][8 * i:8 * i + 8])
                                                           for i in range(n)],
                    "f_ii": list(st["features_ii"])})
    return sizes, e_x, e_b, out


def samples_from_runs(runs):
    """(list of stage samples, list of Stage II samples) from one problem's
    runs.  A sample is (features, a_label, g_label, s_label, w_a, w_s)."""
    ok = [r for r in runs if "error" not in r and r["converged"]]
    if not ok:
        return [], []
    c_min = min(r["cost"] for r in ok)
    near = [r for r in ok if r["cost"] <= COST_TOL * c_min]
    best = max(near, key=lambda r: (r["j"], PATTERN_ORDER[r["pattern"]], r["a"]))
    stage = []
    n = len(best["f_stage"])
    for i in range(n):
        stop = 1 if (best["j"] > 0 and i == len(best["a_list"]) - 1) else 0
        stage.append((best["f_stage"][i], best["a_list"][i], stop, 0.0, 1.0, 0.0))
    ii = [(r["f_ii"], 0, 0, float(r["T2"]), 0.0, 1.0) for r in ok]
    return stage, ii


def to_tensors(samples, device):
    f = torch.tensor([s[0] for s in samples], dtype=torch.float32, device=device).contiguous()
    a = torch.tensor([s[1] for s in samples], dtype=torch.int32, device=device)
    g = torch.tensor([s[2] for s in samples], dtype=torch.int32, device=device)
    s_ = torch.tensor([s[3] for s in samples], dtype=torch.float32, device=device)
    wa = torch.tensor([s[4] for s in samples], dtype=torch.float32, device=device)
    ws = torch.tensor([s[5] for s in samples], dtype=torch.float32, device=device)
    return f, a, g, s_, wa, ws


def train(ctx, data, steps=4000, lr=3e-3, seed=0, W=None, log_every=500, log=None, val=None):
    """Full-batch Adam on the GPU with the library's kernels; the learning
    rate decays linearly to lr/10.  With ``val`` (tensors as ``data``) the
    validation loss is taken every log_every steps and the weights with
    the lowest one are returned (early stopping).  Returns (W, losses),
    losses = [(step, train loss, validation loss or None)]."""
    f, a, g, s_, wa, ws = data
    dev = f.device
    if W is None:
        W = init_weights(seed, dev)
    m = torch.zeros_like(W)
    v = torch.zeros_like(W)
    grad = torch.empty_like(W)
    vgrad = torch.empty_like(W)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    vloss = torch.empty(1, dtype=torch.float32, device=dev)
    losses = []
    best = (float("inf"), W.clone())
    for t in range(1, steps + 1):
        spcg_mlp_loss_grad(ctx, W, f, a, g, s_, wa, ws, grad=grad, loss=loss)
        lr_t = lr * (1.0 - 0.9 * (t - 1) / max(steps - 1, 1))
        spcg_mlp_adam(ctx, W, grad, m, v, t, lr_t)
        if t == 1 or t % log_every == 0 or t == steps:
            vl = None
            if val is not None:
                spcg_mlp_loss_grad(ctx, W, *val, grad=vgrad, loss=vloss)
                vl = float(vloss.item())
                if vl < best[0]:
                    best = (vl, W.clone())
            losses.append((t, float(loss.item()), vl))
            if log:
                log(f"step {t} loss {losses[-1][1]:.5f}" + (f" validation {vl:.5f}" if vl is not None else ""))
    if val is not None:
        W = best[1]
    return W, losses


def predict(ctx, W, feats):
    """(a_i, stop, s_hat) per row of feats (float32 device tensor n x 8)."""
    out = spcg_mlp_forward(ctx, W, feats).cpu().numpy()
    a = out[:, 0:NA].argmax(axis=1)
    stop = out[:, NA:NA + 2].argmax(axis=1)
    return a, stop, out[:, NA + 2] * L.SPCG_MLP_S_SCALE

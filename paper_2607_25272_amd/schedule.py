"""Learned schedule: weights, labels from the method's own runs, training.

The network (three dense FP32 layers, see ``include/spcg.h``) chooses the
Stage I iteration count a, the prefix stride and the number of Stage II
iterations to run before the first stopping test.  Everything here runs
through the library: the labels come from ``spcg_solve`` runs with the
plain schedule, and training calls the library's forward/backward and Adam
kernels (``spcg_mlp_loss_grad``, ``spcg_mlp_adam``) on the GPU.

Labels.  For a problem, the eight variants (a in 1..4) x (stride in 1, 2)
are solved with the plain stopping test.  The variant with the smallest
measured solve time gives the pre-Stage-I sample (features, a - 1,
stride - 1); every variant gives a Stage II sample (its Stage II features,
the Stage II iteration count the plain test chose).
"""
import json
import os

import numpy as np
import torch

from . import _lib as L
from . import spcg_mlp_adam, spcg_mlp_forward, spcg_mlp_loss_grad, spcg_solve

WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedule_weights.json")
VARIANTS = [(a, s) for s in (1, 2) for a in (1, 2, 3, 4)]
PLAIN = (3, 1)


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


def run_variants(ctx, prob, tol=5e-7, seed=1, beta=None):
    """Solves prob with every (a, stride) variant under the plain test.
    Returns a list of dicts (None entries for variants that failed)."""
    if beta is None:
        beta = torch.zeros(prob.d, dtype=torch.float64, device=prob.X.device)
    kw = dict(beta=beta, col_scale=prob.col_scale, seed=seed, tol=tol, record_features=True,
              time_phases=True)
    spcg_solve(ctx, prob.X, prob.Y, a=3, stage_stride=1, **kw)  # workspaces sized, caches warm
    out = []
    for a, stride in VARIANTS:
        try:
            _, st = spcg_solve(ctx, prob.X, prob.Y, a=a, stage_stride=stride, **kw)
        except Exception as e:  # a failing variant gives no label
            out.append({"a": a, "stride": stride, "error": str(e)})
            continue
        out.append({"a": a, "stride": stride, "t_ms": st["t_total_ms"], "T1": st["T_stage1"],
                    "T2": st["T_stage2"], "K": st["K"], "converged": bool(st["converged"]),
                    "syncs": st["host_syncs"], "f_pre": list(st["features_pre"]),
                    "f_ii": list(st["features_ii"])})
    return out


def samples_from_runs(runs):
    """(pre sample or None, list of Stage II samples) from one problem's runs.
    A sample is (features, a_label, g_label, s_label, w_a, w_s)."""
    ok = [r for r in runs if "error" not in r and r["converged"]]
    if not ok:
        return None, []
    best = min(ok, key=lambda r: r["t_ms"])
    pre = (best["f_pre"], best["a"] - 1, best["stride"] - 1, 0.0, 1.0, 0.0)
    ii = [(r["f_ii"], 0, 0, float(r["T2"]), 0.0, 1.0) for r in ok]
    return pre, ii


def to_tensors(samples, device):
    f = torch.tensor([s[0] for s in samples], dtype=torch.float32, device=device).contiguous()
    a = torch.tensor([s[1] for s in samples], dtype=torch.int32, device=device)
    g = torch.tensor([s[2] for s in samples], dtype=torch.int32, device=device)
    s_ = torch.tensor([s[3] for s in samples], dtype=torch.float32, device=device)
    wa = torch.tensor([s[4] for s in samples], dtype=torch.float32, device=device)
    ws = torch.tensor([s[5] for s in samples], dtype=torch.float32, device=device)
    return f, a, g, s_, wa, ws


def train(ctx, data, steps=4000, lr=3e-3, seed=0, W=None, log_every=500, log=None):
    """Full-batch Adam on the GPU with the library's kernels; the learning
    rate decays linearly to lr/10.  Returns (W, losses)."""
    f, a, g, s_, wa, ws = data
    dev = f.device
    if W is None:
        W = init_weights(seed, dev)
    m = torch.zeros_like(W)
    v = torch.zeros_like(W)
    grad = torch.empty_like(W)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    losses = []
    for t in range(1, steps + 1):
        spcg_mlp_loss_grad(ctx, W, f, a, g, s_, wa, ws, grad=grad, loss=loss)
        lr_t = lr * (1.0 - 0.9 * (t - 1) / max(steps - 1, 1))
        spcg_mlp_adam(ctx, W, grad, m, v, t, lr_t)
        if t == 1 or t % log_every == 0 or t == steps:
            losses.append((t, float(loss.item())))
            if log:
                log(f"step {t} loss {losses[-1][1]:.5f}")
    return W, losses


def predict(ctx, W, feats):
    """(a, stride, s_hat) per row of feats (float32 device tensor n x 8)."""
    out = spcg_mlp_forward(ctx, W, feats).cpu().numpy()
    a = out[:, 0:4].argmax(axis=1) + 1
    stride = out[:, 4:6].argmax(axis=1) + 1
    return a, stride, out[:, 6] * L.SPCG_MLP_S_SCALE

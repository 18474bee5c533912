"""GPU checks of the learned schedule.

* The network's forward pass, loss gradient and Adam step (the library's
  HIP kernels, FP32) against the FP64 oracle in ``oracle/mlp.py`` to about
  1e-5 relative, and a short training run against the oracle's trajectory.
* The schedule features computed on the device against the oracle's
  definition on the same inputs: the base and Stage II features, and the
  per-stage features along the oracle's own Stage I trajectory.
* The solve follows the network's per-stage decisions exactly (crafted
  weights; random weights checked stage by stage against the oracle's
  forward pass on the recorded features), stays within 1e-6 of the OLS
  estimator, makes no stream synchronisation in Stage I, and with the
  decisions fixed gives the same bits as the plain schedule with those
  settings.
* The trained weights shipped with the package read fewer bytes in their
  product passes than the plain schedule on the evaluation workload
  (N = 2e6, d = 256, 1% of rows scaled by 100) at equal accuracy.
"""
import os
import statistics
import time

import numpy as np
import pytest
import torch

import workloads
from oracle import mlp
from oracle.ols import ols_tsqr
from oracle.sketch import nested_srht
from oracle.spcg import rel_pred_error, spcg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def S():
    import paper_2607_25272_amd as spcg_mod
    return spcg_mod


@pytest.fixture(scope="module")
def ctx(S):
    c = S.Context(0)
    yield c
    c.close()


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    th = mlp.init(seed) * scale + 0.05 * rng.standard_normal(mlp.n_params())
    return th.astype(np.float32)


def _batch(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, mlp.F)).astype(np.float32)
    a = rng.integers(0, mlp.NA, n).astype(np.int32)
    g = rng.integers(0, 2, n).astype(np.int32)
    s = rng.integers(0, 30, n).astype(np.float32)
    wa = (rng.random(n) < 0.3).astype(np.float32)
    ws = (1.0 - wa).astype(np.float32)
    return X, a, g, s, wa, ws


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(x)).to(DEV) for x in arrs]


@pytest.mark.parametrize("n", [1, 33, 1000, 70_000])
def test_forward_matches_oracle(S, ctx, n):
    th = _rand_params(1)
    X = _batch(n, n)[0]
    W, Xd = _dev(th, X)
    out = S.spcg_mlp_forward(ctx, W, Xd).cpu().numpy()
    ref, _ = mlp.forward(th.astype(np.float64), X.astype(np.float64))
    err = np.abs(out - ref).max() / max(1.0, np.abs(ref).max())
    print(f"forward n={n} max rel err {err:.2e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("n", [1, 31, 32, 33, 5000, 20_000])
def test_loss_grad_matches_oracle(S, ctx, n):
    th = _rand_params(2)
    X, a, g, s, wa, ws = _batch(100 + n, n)
    tens = _dev(th, X, a, g, s, wa, ws)
    grad, loss = S.spcg_mlp_loss_grad(ctx, *tens)
    grad, loss = grad.cpu().numpy().astype(np.float64), float(loss.item())
    lref, gref = mlp.loss_and_grad(th.astype(np.float64), X.astype(np.float64), a, g, s, wa, ws)
    rel = np.linalg.norm(grad - gref) / np.linalg.norm(gref)
    emax = np.abs(grad - gref).max() / np.abs(gref).max()
    print(f"grad n={n}: loss {loss:.6f} vs {lref:.6f}, rel {rel:.2e}, max {emax:.2e}", flush=True)
    assert abs(loss - lref) <= 1e-5 * max(1.0, abs(lref))
    assert rel <= 1e-5 and emax <= 1e-5


def test_loss_grad_is_deterministic(S, ctx):
    th = _rand_params(3)
    tens = _dev(th, *_batch(7, 9000))
    g1, l1 = S.spcg_mlp_loss_grad(ctx, *tens)
    g2, l2 = S.spcg_mlp_loss_grad(ctx, *tens)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_adam_matches_oracle(S, ctx):
    rng = np.random.default_rng(5)
    th = rng.standard_normal(mlp.n_params()).astype(np.float32)
    W, m, v = _dev(th, np.zeros_like(th), np.zeros_like(th))
    t64, m64, v64 = th.astype(np.float64), np.zeros(th.size), np.zeros(th.size)
    for t in range(1, 6):
        gr = rng.standard_normal(th.size).astype(np.float32)
        (G,) = _dev(gr)
        S.spcg_mlp_adam(ctx, W, G, m, v, t, 1e-2)
        t64, m64, v64 = mlp.adam_step(t64, gr.astype(np.float64), m64, v64, t, 1e-2)
    err = np.abs(W.cpu().numpy() - t64).max()
    print(f"adam max abs err {err:.2e}", flush=True)
    assert err <= 1e-6 * max(1.0, np.abs(t64).max())


def test_training_follows_oracle_trajectory(S, ctx):
    # a teacher network labels random features; 60 Adam steps on the GPU
    # kernels and in the FP64 oracle from the same start
    n = 512
    teacher = _rand_params(11, scale=1.5).astype(np.float64)
    X = np.random.default_rng(12).standard_normal((n, mlp.F)).astype(np.float32)
    out, _ = mlp.forward(teacher, X.astype(np.float64))
    a = out[:, 0:4].argmax(1).astype(np.int32)
    g = out[:, 4:6].argmax(1).astype(np.int32)
    s = np.clip(np.rint(out[:, 6] * 3 + 8), 0, 40).astype(np.float32)
    wa = np.ones(n, np.float32)
    ws = np.ones(n, np.float32)
    th0 = _rand_params(13)
    W, m, v, Xd, ad, gd, sd, wad, wsd = _dev(th0, np.zeros_like(th0), np.zeros_like(th0), X, a, g, s, wa, ws)
    t64, m64, v64 = th0.astype(np.float64), np.zeros(th0.size), np.zeros(th0.size)
    l_first = None
    for t in range(1, 61):
        grad, loss = S.spcg_mlp_loss_grad(ctx, W, Xd, ad, gd, sd, wad, wsd)
        S.spcg_mlp_adam(ctx, W, grad, m, v, t, 3e-3)
        l64, g64 = mlp.loss_and_grad(t64, X.astype(np.float64), a, g, s, wa, ws)
        t64, m64, v64 = mlp.adam_step(t64, g64, m64, v64, t, 3e-3)
        if t == 1:
            l_first = l64
    l_gpu = float(S.spcg_mlp_loss_grad(ctx, W, Xd, ad, gd, sd, wad, wsd)[1].item())
    l_ref, _ = mlp.loss_and_grad(t64, X.astype(np.float64), a, g, s, wa, ws)
    print(f"training: loss {l_first:.4f} -> gpu {l_gpu:.5f} / oracle {l_ref:.5f}", flush=True)
    assert l_ref < 0.6 * l_first
    assert abs(l_gpu - l_ref) <= 1e-3 * l_ref
    assert np.abs(W.cpu().numpy() - t64).max() <= 1e-3


@pytest.mark.parametrize("N,d,storage", [(200, 8, "f64"), (1 << 14, 40, "f32"), (30_000, 64, "bf16"),
                                         (30_000, 64, "fp8")])
def test_features_match_oracle(S, ctx, N, d, storage):
    print(f"features N={N} d={d} {storage}", flush=True)
    p = workloads.gauss_colscale(N, d, 1e3, 0.1, storage=storage, seed=N + d, device=DEV,
                                 leverage_frac=0.01)
    beta, st = S.spcg_solve(ctx, p.X, p.Y, col_scale=p.col_scale, seed=4, record_features=True)
    assert st["converged"]
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=4, col_scale=p.col_scale)
    pc = S.spcg_precond_build(ctx, sk)
    R, _ = pc.export()
    rows = mlp.sample_rows(N)
    Xr = p.x_f64(torch.as_tensor(rows, device=DEV)).cpu().numpy()
    f_ref = mlp.features_pre(Xr, N, d, np.diag(R))
    f_gpu = np.array(st["features_pre"], dtype=np.float64)
    assert np.abs(f_gpu - f_ref).max() <= 1e-5, (f_gpu, f_ref)
    fii_ref = mlp.features_ii(f_ref, st["rho_ii0"], st["ax2_ii0"], st["resid2_ii0"], 5e-7)
    fii_gpu = np.array(st["features_ii"], dtype=np.float64)
    assert np.abs(fii_gpu - fii_ref).max() <= 1e-5, (fii_gpu, fii_ref)
    sk.free()
    pc.free()


def test_stage_features_match_oracle_trajectory(S, ctx):
    # cfg0 in FP64: the GPU's Stage I iterates equal the oracle's to 1e-9,
    # so the stage-start residual-to-fit ratios (rows of the nested start
    # pass) agree as well; every stage's features against features_stage
    p = workloads.make_config(0, device=DEV)
    Xd = p.x_f64().cpu().numpy()
    Yd = p.Y.cpu().numpy()[:, 0]
    N, d = Xd.shape
    beta, st = S.spcg_solve(ctx, p.X, p.Y, seed=1, record_features=True)
    assert st["converged"]
    _, info = spcg(Xd, Yd, 1, a=3, nested_gradient=True)
    sizes = info["sizes"]
    K = len(sizes)
    assert st["stages_planned"] == K and list(st["stage_iters"][:K]) == [3] * K
    B, BY, _, _ = nested_srht(Xd, Yd, 1, sizes[-1], 6 * d)
    f_pre = np.array(st["features_pre"], dtype=np.float64)
    stage_x = info["per_rhs"][0]["stage_x"]
    for s_ in range(min(K, 16)):
        lo = sizes[s_ - 1] if s_ > 0 else 0
        x = stage_x[s_ - 1] if s_ > 0 else np.zeros(d)
        fit = B[lo:sizes[s_]] @ x
        res = BY[lo:sizes[s_]] - fit
        f_ref = mlp.features_stage(f_pre, sizes, s_, d, float(res @ res), float(fit @ fit))
        f_gpu = np.array(st["stage_features"][8 * s_:8 * s_ + 8], dtype=np.float64)
        assert np.abs(f_gpu - f_ref).max() <= 1e-5, (s_, f_gpu, f_ref)


def _crafted(b3):
    th = np.zeros(mlp.n_params(), np.float32)
    th[-mlp.O:] = b3
    return torch.from_numpy(th).to(DEV)


@pytest.fixture(scope="module")
def prob0():
    p = workloads.make_config(0, device=DEV)
    Xd = p.x_f64().cpu().numpy()
    return p, Xd, ols_tsqr(Xd, p.Y.cpu().numpy())[:, 0]


# crafted networks: zero weights, so every stage sees outputs = b3
@pytest.mark.parametrize("b3,a,stop,unchecked", [
    ([0, 0, 0, 5, 0, 3, 0, 0.0], 3, 0, 0),      # the plain schedule
    ([0, 0, 7, 0, 0, 0, 4, 0.0], 2, 1, 0),      # a_1 = 2, then Stage II
    ([9, 0, 0, 0, 0, 2, 0, 0.74], 0, 0, 6),     # starts only, 6 unchecked Stage II iterations
    ([0, 0, 0, 0, 3, 0, 1, 0.3], 4, 1, 2),
])
def test_learned_solve_follows_the_network(S, ctx, prob0, b3, a, stop, unchecked):
    p, Xd, bh = prob0
    W = _crafted(b3)
    beta, st = S.spcg_solve(ctx, p.X, p.Y, seed=3, schedule="learned", weights=W)
    K = st["stages_planned"]
    its = list(st["stage_iters"][:K])
    print("learned", b3, its, {k: st[k] for k in ("K", "T_stage1", "T_stage2", "unchecked_iters", "fallback",
                                                  "host_syncs", "s_pred")}, flush=True)
    n = 1 if stop else K
    assert its == [a] * n + [-1] * (K - n)
    assert st["converged"] and st["K"] == n and st["T_stage1"] == a * n
    assert st["unchecked_iters"] == mlp.unchecked_iters(b3[7], 1, 100 - st["T_stage1"]) == unchecked
    assert abs(st["s_pred"] - b3[7] * 10) < 1e-4
    assert rel_pred_error(Xd, beta.cpu().numpy(), bh) <= 1e-6
    # the recorded outputs are the network's, for every started stage
    assert np.allclose(np.array(st["stage_out"][:8 * n]).reshape(n, 8), np.array(b3, np.float32)[None, :])
    # with the same decisions the plain schedule runs the same kernels (the
    # switched-off launches change nothing) and the same host syncs
    plain, stp = S.spcg_solve(ctx, p.X, p.Y, seed=3, a_list=[a] * n, stage_limit=n if stop else 0)
    assert list(stp["stage_iters"][:K]) == its
    if unchecked == 0:
        assert torch.equal(plain, beta)
        assert st["T_stage2"] == stp["T_stage2"] and not st["fallback"]
        assert st["host_syncs"] == stp["host_syncs"]
    else:
        # the first test comes after `unchecked` iterations: never earlier
        assert st["T_stage2"] >= unchecked
        assert st["fallback"] == int(stp["T_stage2"] > unchecked)


def test_learned_stage_one_respects_the_budget(S, ctx, prob0):
    # a = 4 at every stage with T = 7: Stage I takes T - 1 = 6 iterations
    # (4, then 2, then 0 per stage) and Stage II is left one
    p = prob0[0]
    W = _crafted([0, 0, 0, 0, 5, 1, 0, 0.0])
    _, st = S.spcg_solve(ctx, p.X, p.Y, seed=3, schedule="learned", weights=W, T=7)
    K = st["stages_planned"]
    assert list(st["stage_iters"][:K]) == [4, 2] + [0] * (K - 2)
    assert st["T_stage1"] == 6 and st["T_stage2"] <= 1


@pytest.mark.parametrize("seed", [0, 1])
def test_learned_decisions_match_oracle_forward(S, ctx, seed):
    # random networks: at every started stage the device decision equals
    # the oracle's policy on the recorded features, and the recorded
    # outputs equal the oracle's forward pass on them
    p = workloads.gauss_colscale(60_000, 24, 1e4, 0.1, storage="f32", seed=70 + seed, device=DEV)
    th = _rand_params(seed, scale=0.3)
    # bias the stop logits so that Stage I does not stop at once
    th[-3] += 1.0
    W = torch.from_numpy(th).to(DEV)
    _, st = S.spcg_solve(ctx, p.X, p.Y, seed=2, schedule="learned", weights=W)
    K = st["stages_planned"]
    its = list(st["stage_iters"][:K])
    started = [i for i in range(K) if its[i] >= 0]
    print(f"random network {seed}: K={K} iters={its}", flush=True)
    assert started == list(range(len(started))) and started
    for i in started[:16]:
        f = np.array(st["stage_features"][8 * i:8 * i + 8], np.float64)
        out_ref, _ = mlp.forward(th.astype(np.float64), f[None, :])
        out_gpu = np.array(st["stage_out"][8 * i:8 * i + 8], np.float64)
        assert np.abs(out_gpu - out_ref[0]).max() <= 1e-4 * max(1.0, np.abs(out_ref).max())
        a_i, stop = mlp.policy_stage(out_gpu)
        assert its[i] == a_i
        if i < K - 1:   # the last planned stage's stop decision has no effect
            assert stop == int(i == started[-1])


def test_learned_rejects_bad_use(S, ctx, prob0):
    p = prob0[0]
    with pytest.raises(S.SpcgError):
        S.spcg_solve(ctx, p.X, p.Y, schedule="learned")
    with pytest.raises(S.SpcgError):
        S.spcg_solve(ctx, p.X, p.Y, schedule="learned", weights=_crafted([0] * 8), method="pcg")


WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2607_25272_amd",
                       "schedule_weights.json")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights shipped")
def test_trained_schedule_reads_fewer_bytes_on_high_leverage_workload(S, ctx):
    # count-based: the bytes the product passes read (schedule.solve_cost)
    # at equal accuracy; the times are printed, not asserted
    from paper_2607_25272_amd import schedule
    W = schedule.load_weights(DEV)
    p = workloads.make_config(4, device=DEV)
    print(f"gain workload N={p.N} d={p.d}", flush=True)
    sizes, e_x, e_b = schedule.problem_sizes(ctx, p)
    beta = torch.zeros(p.d, dtype=torch.float64, device=DEV)
    Xd = p.x_f64().cpu().numpy()
    bh = ols_tsqr(Xd, p.Y.cpu().numpy())[:, 0]
    res = {}
    for name in ("plain", "learned"):
        kw = dict(schedule="learned", weights=W) if name == "learned" else {}
        S.spcg_solve(ctx, p.X, p.Y, beta=beta, seed=1, **kw)
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = S.spcg_solve(ctx, p.X, p.Y, beta=beta, seed=1, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        err = rel_pred_error(Xd, beta.cpu().numpy(), bh)
        cost = schedule.solve_cost(st, sizes, p.N, p.d, e_x, e_b)
        res[name] = (cost, statistics.median(ts) * 1e3, st)
        K = st["stages_planned"]
        print(f"{name}: {cost / 1e9:.3f} GB read, {res[name][1]:.3f} ms, iters {list(st['stage_iters'][:K])} "
              f"T2={st['T_stage2']} syncs={st['host_syncs']} rel={err:.2e}", flush=True)
        assert st["converged"] and err <= 1e-6
    print(f"gain: bytes plain/learned = {res['plain'][0] / res['learned'][0]:.3f}, "
          f"time plain/learned = {res['plain'][1] / res['learned'][1]:.3f}", flush=True)
    assert res["learned"][0] < res["plain"][0]
    assert res["learned"][2]["host_syncs"] <= res["plain"][2]["host_syncs"]
